// Host-side split of a grouped SGEMM launch's tiles over the 8 XCDs by work
// (no HIP types; a CPU test checks it).
#pragma once

#include <algorithm>
#include <cstdint>

namespace gvm {

// Work of one tile in k-steps: its k-loop plus a fixed part for the prologue
// and the store of C (about four k-steps).
inline uint64_t gemm_tile_work(uint32_t ksteps) { return static_cast<uint64_t>(ksteps) + 4; }

// Requests i = 0 .. count-1 hold units[i] tiles of ksteps[i] k-steps each,
// numbered consecutively from 0.  Writes begin[0..8]: XCD x takes the units
// [begin[x], begin[x + 1]), where begin[x] (x = 1..7) is the first unit at
// whose start the work of the units before it reaches x / 8 of the total
// (rounded up); begin[0] = 0, begin[8] = the number of units, and begin is
// non-decreasing.
inline void balance_xcd_runs(uint32_t count, const uint32_t* units, const uint32_t* ksteps, uint32_t begin[9]) {
  uint64_t total = 0;
  uint32_t all = 0;
  for (uint32_t i = 0; i < count; ++i) {
    total += static_cast<uint64_t>(units[i]) * gemm_tile_work(ksteps[i]);
    all += units[i];
  }
  begin[0] = 0;
  uint64_t before = 0;  // work of the requests before request i
  uint32_t first = 0;   // first unit of request i
  uint32_t i = 0;
  for (int x = 1; x < 8; ++x) {
    const uint64_t target = (total * static_cast<uint64_t>(x) + 7) / 8;
    while (i < count && before + static_cast<uint64_t>(units[i]) * gemm_tile_work(ksteps[i]) <= target) {
      before += static_cast<uint64_t>(units[i]) * gemm_tile_work(ksteps[i]);
      first += units[i];
      ++i;
    }
    uint32_t cut = all;
    if (i < count) {
      const uint64_t w = gemm_tile_work(ksteps[i]);
      cut = first + static_cast<uint32_t>((target - before + w - 1) / w);
    }
    begin[x] = std::max(begin[x - 1], std::min(cut, all));
  }
  begin[8] = all;
}

}  // namespace gvm
