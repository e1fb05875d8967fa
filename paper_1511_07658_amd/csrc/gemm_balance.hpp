// Host-side split of a grouped SGEMM launch's tiles over the 8 XCDs by work
// (no HIP types; a CPU test checks it).
#pragma once

#include <algorithm>
#include <cstdint>

namespace gvm {

// Work of one tile in k-steps: its k-loop plus a fixed part for the prologue
// and the store of C (about four k-steps).
inline uint64_t gemm_tile_work(uint32_t ksteps) { return static_cast<uint64_t>(ksteps) + 4; }

constexpr int kGemmSlices = 16;  // slices of equal work, two per XCD

// Requests i = 0 .. count-1 hold units[i] tiles of ksteps[i] k-steps each,
// numbered consecutively from 0 (largest requests first).  Writes
// cut[0..kGemmSlices]: slice s is the units [cut[s], cut[s + 1]), where
// cut[s] (s = 1 .. kGemmSlices - 1) is the first unit at whose start the work
// of the units before it reaches s / kGemmSlices of the total (rounded up);
// cut[0] = 0, cut[kGemmSlices] = the number of units, and cut is
// non-decreasing.
inline void balance_slices(uint32_t count, const uint32_t* units, const uint32_t* ksteps,
                           uint32_t cut[kGemmSlices + 1]) {
  uint64_t total = 0;
  uint32_t all = 0;
  for (uint32_t i = 0; i < count; ++i) {
    total += static_cast<uint64_t>(units[i]) * gemm_tile_work(ksteps[i]);
    all += units[i];
  }
  cut[0] = 0;
  uint64_t before = 0;  // work of the requests before request i
  uint32_t first = 0;   // first unit of request i
  uint32_t i = 0;
  for (int s = 1; s < kGemmSlices; ++s) {
    const uint64_t target = (total * static_cast<uint64_t>(s) + kGemmSlices - 1) / kGemmSlices;
    while (i < count && before + static_cast<uint64_t>(units[i]) * gemm_tile_work(ksteps[i]) <= target) {
      before += static_cast<uint64_t>(units[i]) * gemm_tile_work(ksteps[i]);
      first += units[i];
      ++i;
    }
    uint32_t c = all;
    if (i < count) {
      const uint64_t w = gemm_tile_work(ksteps[i]);
      c = first + static_cast<uint32_t>((target - before + w - 1) / w);
    }
    cut[s] = std::max(cut[s - 1], std::min(c, all));
  }
  cut[kGemmSlices] = all;
}

// The two slices XCD x (0..7) works through, in order.  Contiguous: slices
// 2x and 2x + 1 (one run of an eighth of the work).  Paired: slice x from the
// long end and slice 15 - x from the short end, so that every XCD starts on
// long tiles and ends on short ones and no XCD's last tiles are long ones.
inline void xcd_slices(int x, bool paired, int* first, int* second) {
  if (paired) {
    *first = x;
    *second = kGemmSlices - 1 - x;
  } else {
    *first = 2 * x;
    *second = 2 * x + 1;
  }
}

}  // namespace gvm
