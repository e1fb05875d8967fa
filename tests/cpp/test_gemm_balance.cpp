// CPU check of the SGEMM launch's split over XCDs (csrc/gemm_balance.hpp):
// for random groups of requests, the runs cover every unit once, each run's
// work is within one tile of an eighth of the total, and the kernel's index
// walk over the balanced grid (XCD x = workgroup % 8, one workgroup per unit
// of the longest run) visits every unit exactly once and none beyond.
#include <cstdio>
#include <random>
#include <vector>

#include "gemm_balance.hpp"

static int failures = 0;
#define CHECK(c, ...)                  \
  do {                                 \
    if (!(c)) {                        \
      ++failures;                      \
      printf("FAIL: " __VA_ARGS__);    \
      printf("\n");                    \
    }                                  \
  } while (0)

static void check_group(const std::vector<uint32_t>& units, const std::vector<uint32_t>& ksteps) {
  const uint32_t count = static_cast<uint32_t>(units.size());
  uint32_t begin[9];
  gvm::balance_xcd_runs(count, units.data(), ksteps.data(), begin);
  std::vector<uint64_t> work_at;  // work of the units before unit u
  uint64_t total = 0, wmax = 0;
  for (uint32_t i = 0; i < count; ++i)
    for (uint32_t t = 0; t < units[i]; ++t) {
      work_at.push_back(total);
      total += gvm::gemm_tile_work(ksteps[i]);
      wmax = std::max<uint64_t>(wmax, gvm::gemm_tile_work(ksteps[i]));
    }
  const uint32_t all = static_cast<uint32_t>(work_at.size());
  work_at.push_back(total);
  CHECK(begin[0] == 0 && begin[8] == all, "ends %u %u of %u", begin[0], begin[8], all);
  uint32_t most = 0;
  for (int x = 0; x < 8; ++x) {
    CHECK(begin[x] <= begin[x + 1], "run %d decreasing", x);
    const uint64_t w = work_at[begin[x + 1]] - work_at[begin[x]];
    const double share = total / 8.0;
    CHECK(w <= share + wmax + 1 && w + wmax + 1 >= share, "run %d work %llu, eighth %.1f, tile %llu", x,
          (unsigned long long)w, share, (unsigned long long)wmax);
    most = std::max(most, begin[x + 1] - begin[x]);
  }
  // the kernel's walk: grid = 8 * most, u = begin[x] + j, step most
  std::vector<int> seen(all, 0);
  const uint32_t grid = 8 * most;
  for (uint32_t w = 0; w < grid; ++w) {
    const uint32_t x = w % 8;
    for (uint32_t u = begin[x] + w / 8; u < begin[x + 1]; u += grid / 8) {
      CHECK(u < all, "unit %u beyond %u", u, all);
      if (u < all) ++seen[u];
    }
  }
  for (uint32_t u = 0; u < all; ++u) CHECK(seen[u] == 1, "unit %u visited %d times", u, seen[u]);
}

int main() {
  // the 16 uneven sizes of the 32-rank batch, 64x128 tiles of BK = 16, largest first
  const uint32_t sizes[] = {1920, 1728, 1664, 1408, 1280, 1280, 1216, 1216, 960, 832, 832, 704, 704, 704, 448, 384};
  std::vector<uint32_t> u, k;
  for (uint32_t n : sizes) {
    u.push_back(((n + 63) / 64) * ((n + 127) / 128));
    k.push_back((n + 15) / 16);
  }
  check_group(u, k);
  std::mt19937 g(1511);
  for (int t = 0; t < 20000; ++t) {
    const uint32_t count = 1 + g() % 32;
    std::vector<uint32_t> uu, kk;
    for (uint32_t i = 0; i < count; ++i) {
      uu.push_back(g() % 5 == 0 ? 1 + g() % 3 : 1 + g() % 900);
      kk.push_back(1 + g() % 256);
    }
    check_group(uu, kk);
  }
  check_group({1}, {1});
  check_group({3, 1}, {7, 1});
  printf("ok: %d failures\n", failures);
  return failures ? 1 : 0;
}
