// CPU check of the SGEMM launch's split over XCDs (csrc/gemm_balance.hpp):
// for random groups of requests, the 16 slices cover every unit once, each
// slice's work is within one tile of a sixteenth of the total, and the
// kernel's index walk over the balanced grid (XCD x = workgroup % 8, its two
// slices from xcd_slices, one workgroup per unit of the longest pair) visits
// every unit exactly once and none beyond, for both slice pairings.
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
  uint32_t cut[gvm::kGemmSlices + 1];
  gvm::balance_slices(count, units.data(), ksteps.data(), cut);
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
  CHECK(cut[0] == 0 && cut[gvm::kGemmSlices] == all, "ends %u %u of %u", cut[0], cut[gvm::kGemmSlices], all);
  for (int s = 0; s < gvm::kGemmSlices; ++s) {
    CHECK(cut[s] <= cut[s + 1], "slice %d decreasing", s);
    const uint64_t w = work_at[cut[s + 1]] - work_at[cut[s]];
    const double share = total / double(gvm::kGemmSlices);
    CHECK(w <= share + wmax + 1 && w + wmax + 1 >= share, "slice %d work %llu, share %.1f, tile %llu", s,
          (unsigned long long)w, share, (unsigned long long)wmax);
  }
  for (int paired = 0; paired < 2; ++paired) {
    // every slice belongs to exactly one XCD
    std::vector<int> owner(gvm::kGemmSlices, 0);
    uint32_t most = 0;
    for (int x = 0; x < 8; ++x) {
      int s0, s1;
      gvm::xcd_slices(x, paired, &s0, &s1);
      ++owner[s0];
      ++owner[s1];
      most = std::max(most, (cut[s0 + 1] - cut[s0]) + (cut[s1 + 1] - cut[s1]));
    }
    for (int s = 0; s < gvm::kGemmSlices; ++s) CHECK(owner[s] == 1, "slice %d owned %d times", s, owner[s]);
    // the kernel's walk: grid = 8 * most, one unit per workgroup
    std::vector<int> seen(all, 0);
    const uint32_t grid = 8 * most;
    for (uint32_t w = 0; w < grid; ++w) {
      const int x = static_cast<int>(w % 8);
      const int s0 = paired ? x : 2 * x;
      const int s1 = paired ? gvm::kGemmSlices - 1 - x : 2 * x + 1;
      int h0, h1;
      gvm::xcd_slices(x, paired, &h0, &h1);
      CHECK(h0 == s0 && h1 == s1, "kernel slices differ from xcd_slices at x %d", x);
      const uint32_t j = w / 8;
      const uint32_t len0 = cut[s0 + 1] - cut[s0];
      const uint32_t u0 = j < len0 ? cut[s0] + j : cut[s1] + (j - len0);
      const uint32_t uend = j < len0 ? cut[s0 + 1] : cut[s1 + 1];
      for (uint32_t u = u0; u < uend; u += uend) {
        CHECK(u < all, "unit %u beyond %u", u, all);
        if (u < all) ++seen[u];
      }
    }
    for (uint32_t u = 0; u < all; ++u) CHECK(seen[u] == 1, "paired %d: unit %u visited %d times", paired, u, seen[u]);
  }
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
