// Concurrency stress of the manager's host protocol on the loopback backend,
// built with the compiler's address/undefined-behaviour or thread sanitizer
// (tests/test_host_sanitizers.py).  No GPU: the loopback device copies each
// request's first output-sized bytes of input to its output (zero-padded),
// so every rank can check that it got its own bytes back through shared
// memory, staging, the "device" slot and the result path.
//
// One process holds the manager (service thread, staging-copy pool) and
// `ranks` rank threads.  Each rank submits a seeded random sequence of
// requests of every kernel id: copy-in and zero-copy inputs, results into
// caller memory or into its own shared-memory space, blocking and
// non-blocking submission, and waits for one ticket, for any ticket or for
// all.  A statistics reader polls gvm_stats_json meanwhile.  Sizes reach
// several copy pieces (GVM_PIECE_MB=1 is set by the caller).
//
//   host_stress <mode 0 batch | 1 serving> <policy 0..3> <ranks> <requests per rank> <seed>
#include <unistd.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "gvm.h"

namespace {

struct Sizes {
  uint64_t in_bytes, out_bytes;
};

Sizes sizes_of(int k, uint64_t n) {
  switch (k) {
    case GVM_K_VECADD:
    case GVM_K_VECMUL:
      return {8 * n, 4 * n};
    case GVM_K_BLACKSCHOLES:
      return {12 * n, 8 * n};
    case GVM_K_SGEMM:
      return {8 * n * n, 4 * n * n};
    default:
      return {16, 96};  // EP: a 128-bit key in, a 12-word record out
  }
}

// Expected loopback result: the first out_bytes of the input, zero-padded.
bool check(const uint8_t* in, const Sizes& s, const uint8_t* out) {
  const uint64_t keep = s.in_bytes < s.out_bytes ? s.in_bytes : s.out_bytes;
  if (memcmp(in, out, keep) != 0) return false;
  for (uint64_t i = keep; i < s.out_bytes; ++i)
    if (out[i]) return false;
  return true;
}

std::atomic<int> failures{0};

void report(int rank, const char* what, long long v) {
  failures.fetch_add(1);
  fprintf(stderr, "rank %d: %s (%lld): %s\n", rank, what, v, gvm_last_error());
}

struct Req {
  int kernel;
  uint64_t n;
  Sizes s;
  std::vector<uint8_t> in, out;
  uint8_t* out_ptr = nullptr;  // caller memory or the rank's shared space
  int64_t ticket = -1;
  bool done = false;
};

uint64_t draw_n(std::mt19937_64& g, int k) {
  switch (k) {
    case GVM_K_VECADD:
    case GVM_K_VECMUL:
      return 1 + g() % (3u << 18);    // up to 6 MiB of input: several 1 MiB pieces
    case GVM_K_BLACKSCHOLES:
      return 1 + g() % (1u << 18);
    case GVM_K_SGEMM:
      return 1 + g() % 700;
    default:
      return 1 + g() % (1u << 20);
  }
}

void rank_body(const char* ns, int rank, int requests, uint64_t seed, uint64_t shm_bytes) {
  int rc = gvm_attach_ns(ns, rank);
  if (rc != GVM_OK) return report(rank, "attach", rc);
  std::mt19937_64 g(seed * 1000003u + static_cast<uint64_t>(rank));
  const int kernels[5] = {GVM_K_VECADD, GVM_K_BLACKSCHOLES, GVM_K_SGEMM, GVM_K_VECMUL, GVM_K_EP};
  std::vector<Req> live;
  int submitted = 0;
  while (submitted < requests || !live.empty()) {
    // submit up to three requests, then wait in one of three ways
    while (submitted < requests && live.size() < 3) {
      Req r;
      r.kernel = kernels[g() % 5];
      r.n = draw_n(g, r.kernel);
      r.s = sizes_of(r.kernel, r.n);
      if (3 * (r.s.in_bytes + r.s.out_bytes) > shm_bytes) continue;
      r.in.resize(r.s.in_bytes);
      for (auto& b : r.in) b = static_cast<uint8_t>(g());
      r.out.assign(r.s.out_bytes, 0xEE);
      r.out_ptr = r.out.data();
      const void* in = r.in.data();
      const unsigned how = static_cast<unsigned>(g() % 4);
      if (how == 1 && live.empty()) {
        // zero-copy: the input and the result in the rank's own space
        auto* buf = static_cast<uint8_t*>(gvm_rank_buffer(rank, r.s.in_bytes + r.s.out_bytes));
        if (buf) {
          memcpy(buf, r.in.data(), r.s.in_bytes);
          in = buf;
          r.out_ptr = buf + r.s.in_bytes;
        }
      }
      const uint32_t flags = (how == 2) ? GVM_F_NONBLOCK : 0u;
      int64_t t;
      while ((t = gvm_submit_ex(rank, r.kernel, in, r.out_ptr, r.n, flags)) == GVM_EAGAIN) usleep(50);
      if (t < 0) {
        report(rank, "submit", t);
        break;
      }
      r.ticket = t;
      live.push_back(std::move(r));
      ++submitted;
      if (in != live.back().in.data()) break;  // zero-copy space in use: wait before the next
    }
    if (live.empty()) break;
    const unsigned w = static_cast<unsigned>(g() % 3);
    if (w == 0) {
      int64_t t = -1;
      rc = gvm_wait_any(rank, 30'000'000'000LL, &t);
      if (rc != GVM_OK) return report(rank, "wait_any", rc);
      for (auto& r : live)
        if (r.ticket == t) r.done = true;
    } else if (w == 1) {
      rc = gvm_wait(rank, live.front().ticket, 30'000'000'000LL);
      if (rc != GVM_OK) return report(rank, "wait", rc);
      live.front().done = true;
    } else {
      rc = gvm_wait(rank, -1, 30'000'000'000LL);
      if (rc != GVM_OK) return report(rank, "wait all", rc);
      for (auto& r : live) r.done = true;
    }
    std::vector<Req> keep;
    for (auto& r : live) {
      if (!r.done) {
        keep.push_back(std::move(r));
        continue;
      }
      if (!check(r.in.data(), r.s, r.out_ptr)) report(rank, "result bytes differ, kernel", r.kernel);
    }
    live.swap(keep);
  }
  rc = gvm_detach(rank);
  if (rc != GVM_OK) report(rank, "detach", rc);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 6) {
    fprintf(stderr, "usage: %s mode policy ranks requests seed\n", argv[0]);
    return 2;
  }
  const int mode = atoi(argv[1]), policy = atoi(argv[2]), ranks = atoi(argv[3]), requests = atoi(argv[4]);
  const uint64_t seed = strtoull(argv[5], nullptr, 10);
  gvm_config cfg;
  gvm_config_default(&cfg);
  cfg.nranks = static_cast<uint32_t>(ranks);
  cfg.shm_bytes_per_rank = 24ull << 20;
  cfg.hbm_budget_bytes = 64ull << 20;  // tight: admission binds in serving mode
  cfg.mode = static_cast<uint32_t>(mode);
  cfg.policy = static_cast<uint32_t>(policy);
  cfg.batch_window_us = 300;
  cfg.max_inflight = static_cast<uint32_t>(ranks / 2 + 1);
  cfg.backend = GVM_BACKEND_LOOPBACK;
  cfg.copy_threads = 3;
  snprintf(cfg.name, sizeof(cfg.name), "gvm.stress.%d", static_cast<int>(getpid()));
  int rc = gvm_init(&cfg);
  if (rc != GVM_OK) {
    fprintf(stderr, "gvm_init: %d %s\n", rc, gvm_last_error());
    return 1;
  }
  std::atomic<bool> stop{false};
  std::thread stats([&] {
    std::vector<char> buf(1 << 16);
    while (!stop.load()) {
      if (gvm_stats_json(buf.data(), buf.size()) < 0) report(-1, "stats", 0);
      usleep(2000);
    }
  });
  std::vector<std::thread> ts;
  for (int r = 0; r < ranks; ++r)
    ts.emplace_back(rank_body, cfg.name, r, requests, seed, static_cast<uint64_t>(cfg.shm_bytes_per_rank));
  for (auto& t : ts) t.join();
  stop.store(true);
  stats.join();
  rc = gvm_shutdown();
  if (rc != GVM_OK) report(-1, "shutdown", rc);
  printf("host stress mode %d policy %d ranks %d requests %d: %d failures\n", mode, policy, ranks, requests,
         failures.load());
  return failures.load() ? 1 : 0;
}
