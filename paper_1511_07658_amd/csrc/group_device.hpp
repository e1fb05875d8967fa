// Device-side helpers shared by the grouped kernels (hipcc only).
#pragma once

#include "kernels.hpp"

namespace gvm {

constexpr int kThreads = 256;   // workgroup size of the streaming kernels
constexpr int kXcds = kGroupXcds;  // MI355X: workgroup w is dispatched to XCD w % 8

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Index of the request whose units contain unit u: the last descriptor with
// unit_begin <= u (descriptors are in unit order, the first starts at 0).
template <class G>
__device__ __forceinline__ int find_request(const G& g, uint64_t u) {
  int lo = 0, hi = static_cast<int>(g.count) - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (g.d[mid].unit_begin <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Launch `kernel(g)` on `s` (nothing for an empty grid).
template <class G>
hipError_t launch_group(void (*kernel)(G), int grid, int block, hipStream_t s, const G& g) {
  if (grid <= 0) return hipSuccess;
  void* args[] = {const_cast<G*>(&g)};
  return hipLaunchKernel(reinterpret_cast<const void*>(kernel), dim3(grid), dim3(block), args, 0, s);
}

}  // namespace gvm
