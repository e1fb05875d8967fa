#include "common.hpp"

#include <atomic>

#include <errno.h>
#include <linux/futex.h>
#include <signal.h>
#include <stdarg.h>
#include <sys/syscall.h>
#include <time.h>
#include <unistd.h>

#include <climits>
#include <cstdlib>
#include <cstring>

namespace gvm {

namespace {
thread_local char t_err[512] = {0};
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_err, sizeof(t_err), fmt, ap);
  va_end(ap);
  return code;
}

const char* last_error_text() { return t_err; }
void clear_error() { t_err[0] = 0; }

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return static_cast<uint64_t>(ts.tv_sec) * 1000000000ull + static_cast<uint64_t>(ts.tv_nsec);
}

bool request_layout(int kernel_id, uint64_t n, Layout* out) {
  if (n == 0) return false;
  const uint64_t f = sizeof(float);
  switch (kernel_id) {
    case GVM_K_VECADD:
    case GVM_K_VECMUL:
      if (n > (1ull << 40)) return false;
      out->in_bytes = 2 * n * f;
      out->out_bytes = n * f;
      return true;
    case GVM_K_BLACKSCHOLES:
      if (n > (1ull << 40)) return false;
      out->in_bytes = 3 * n * f;
      out->out_bytes = 2 * n * f;
      return true;
    case GVM_K_SGEMM:
      if (n > 65536) return false;  // C must fit 32-bit row/col indexing
      out->in_bytes = 2 * n * n * f;
      out->out_bytes = n * n * f;
      return true;
    case GVM_K_EP:
      if (n > (1ull << 40)) return false;
      out->in_bytes = 2 * sizeof(uint64_t);
      out->out_bytes = kEpWords * sizeof(uint64_t);
      out->scratch_bytes = ((n + kEpUnit - 1) / kEpUnit) * kEpWords * sizeof(uint64_t);  // one partial per unit
      return true;
    default:
      return false;
  }
}

namespace {
std::atomic<uint64_t> g_piece_bytes{8ull << 20};
}  // namespace

void set_piece_bytes(uint64_t bytes) { g_piece_bytes.store(bytes, std::memory_order_relaxed); }

uint64_t piece_bytes() {
  static const uint64_t env = [] {
    const char* e = getenv("GVM_PIECE_MB");
    const long mb = e ? atol(e) : 0;
    return mb >= 1 && mb <= 64 ? static_cast<uint64_t>(mb) << 20 : uint64_t(0);
  }();
  return env ? env : g_piece_bytes.load(std::memory_order_relaxed);
}

int cu_partition_masks(uint32_t latency_cus, uint32_t* latency_mask, uint32_t* bulk_mask) {
  if (latency_cus == 0 || latency_cus % 32 || latency_cus >= static_cast<uint32_t>(kPartitionCus)) return GVM_EINVAL;
  const uint32_t m = latency_cus / 32, full = m / 2;
  const bool half = m % 2 != 0;
  for (int w = 0; w < kPartitionCus / 32; ++w) latency_mask[w] = bulk_mask[w] = 0;
  for (uint32_t i = 0; i < static_cast<uint32_t>(kPartitionCus); ++i) {
    const uint32_t a = i / 32, b = (i / 8) % 4, c = i % 8;
    const bool lat = b < full || (half && b == full && (a + c) % 2 == 0);
    (lat ? latency_mask : bulk_mask)[i / 32] |= 1u << (i % 32);
  }
  return GVM_OK;
}

int futex_wait(std::atomic<uint32_t>* word, uint32_t expected, int64_t timeout_ns) {
  timespec ts;
  timespec* tp = nullptr;
  if (timeout_ns >= 0) {
    ts.tv_sec = timeout_ns / 1000000000ll;
    ts.tv_nsec = timeout_ns % 1000000000ll;
    tp = &ts;
  }
  long rc = syscall(SYS_futex, reinterpret_cast<uint32_t*>(word), FUTEX_WAIT, expected, tp, nullptr, 0);
  if (rc == -1 && errno == ETIMEDOUT) return GVM_ETIMEDOUT;
  return 0;
}

void futex_wake_all(std::atomic<uint32_t>* word) {
  syscall(SYS_futex, reinterpret_cast<uint32_t*>(word), FUTEX_WAKE, INT_MAX, nullptr, nullptr, 0);
}

uint64_t spin_env_ns(const char* var, uint64_t default_us) {
  uint64_t us = default_us;
  if (const char* e = getenv(var)) us = strtoull(e, nullptr, 10);
  if (us > 100000) us = 100000;
  return us * 1000ull;
}

bool pid_alive(int32_t pid) {
  if (pid <= 0) return false;
  if (kill(pid, 0) != 0 && errno != EPERM) return false;
  // an exited but unreaped process (zombie) still answers kill(pid, 0)
  char path[64];
  snprintf(path, sizeof(path), "/proc/%d/stat", pid);
  FILE* f = fopen(path, "r");
  if (!f) return true;
  char buf[512];
  size_t len = fread(buf, 1, sizeof(buf) - 1, f);
  fclose(f);
  buf[len] = 0;
  const char* rp = strrchr(buf, ')');
  if (rp && rp[1] == ' ' && (rp[2] == 'Z' || rp[2] == 'X')) return false;
  return true;
}

}  // namespace gvm
