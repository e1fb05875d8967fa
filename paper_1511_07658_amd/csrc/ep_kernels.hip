// EP-like compute-intensive kernel of the GVM for gfx950: the paper's small
// compute-intensive benchmark (NPB EP, Table 3, Section 6) in the form given
// in the public header: Gaussian pairs by Marsaglia's polar method from the
// counter-based generator Philox4x64-10 (Salmon et al., SC 2011), reduced to
// two binary64 sums and ten annulus counts.
//
// A request of n pairs is cut into work units of kEpUnit pairs (the cut
// depends on n only).  One grouped persistent launch computes every unit of
// every request of the group and writes a partial record per unit into the
// request's device scratch; a second launch, one workgroup per request, sums
// the partials in unit order.  Both sums run in a fixed order (per thread in
// block order, then a fixed tree), so a request's result is bit-identical
// alone and in any mix.  Counts are integers and order-free.
#include "common.hpp"
#include "group_device.hpp"

#include <algorithm>

namespace gvm {

namespace {

constexpr int kEpThreads = 256;
constexpr int kEpGrid = 1024;   // persistent grid of the unit launch
static_assert(kEpUnit / kEpThreads <= 255, "per-thread 8-bit annulus counts of a unit would overflow");

// Philox4x64 multipliers and Weyl key increments (Salmon et al., 2011).
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// Philox4x64 with 10 rounds of counter (b, 0, 0, 0) under key (k0, k1): per
// round the full 128-bit products of words 0 and 2 with the multipliers;
// the next counter is (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)); the key is bumped by the Weyl increments between rounds.
__device__ __forceinline__ void philox_block(uint64_t b, uint64_t k0, uint64_t k1, uint64_t w[4]) {
  uint64_t c0 = b, c1 = 0, c2 = 0, c3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  w[0] = c0;
  w[1] = c1;
  w[2] = c2;
  w[3] = c3;
}

// A thread's annulus counts within one work unit, 8 bits each: counts 0..7
// in `lo`, 8..9 in `hi` (a thread tallies at most 2 * kEpUnit / (2 *
// kEpThreads) = 128 pairs of a unit, so no field overflows).
struct Tally {
  uint64_t lo = 0, hi = 0;
  __device__ __forceinline__ void add(int l) {  // l in 0..9, or >= 10: not counted
    const uint64_t one = 1ull << (8 * (l & 7));
    lo += l < 8 ? one : 0;
    hi += (l >= 8 && l < 10) ? one : 0;
  }
  __device__ __forceinline__ uint32_t get(int l) const {
    return static_cast<uint32_t>(((l < 8 ? lo : hi) >> (8 * (l & 7))) & 0xFF);
  }
};

// One pair from two generator words: accept it when 0 < t <= 1 and add its
// Gaussian pair to the running sums and annulus counts.
__device__ __forceinline__ void ep_pair(uint64_t wx, uint64_t wy, double& sx, double& sy, Tally& q) {
#pragma clang fp contract(off)
  const double x = 2.0 * (static_cast<double>(wx >> 11) * 0x1.0p-53) - 1.0;
  const double y = 2.0 * (static_cast<double>(wy >> 11) * 0x1.0p-53) - 1.0;
  const double t = x * x + y * y;  // two rounded products, one rounded sum
  if (t > 0.0 && t <= 1.0) {
    const double f = sqrt(-2.0 * log(t) / t);
    const double X = x * f, Y = y * f;
    sx += X;
    sy += Y;
    const double m = fmax(fabs(X), fabs(Y));
    q.add(m < 10.0 ? static_cast<int>(m) : 10);  // floor for m >= 0
  }
}

// Fixed-order workgroup sum of one value per thread (binary tree over
// thread indices); the result is valid in thread 0.
__device__ __forceinline__ double tree_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = kEpThreads / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kEpThreads) void ep_units_kernel(EpGroup g) {
  __shared__ double red[kEpThreads];
  __shared__ uint32_t cnt[10];
  for (uint64_t u = blockIdx.x; u < g.total_units; u += gridDim.x) {
    const int r = find_request(g, u);
    const EpDesc& d = g.d[r];
    const uint64_t local = u - d.unit_begin;
    const uint64_t p0 = local * kEpUnit;                     // first pair (even)
    const uint64_t p1 = min(p0 + kEpUnit, d.n);              // end of pairs
    const uint64_t k0 = d.key[0], k1 = d.key[1];
    double sx = 0.0, sy = 0.0;
    Tally q;
    if (threadIdx.x < 10) cnt[threadIdx.x] = 0;
    for (uint64_t b = p0 / 2 + threadIdx.x; 2 * b < p1; b += kEpThreads) {
      uint64_t w[4];
      philox_block(b, k0, k1, w);
      ep_pair(w[0], w[1], sx, sy, q);
      if (2 * b + 1 < p1) ep_pair(w[2], w[3], sx, sy, q);
    }
    __syncthreads();  // cnt cleared
#pragma unroll
    for (int l = 0; l < 10; ++l)
      if (q.get(l)) atomicAdd(&cnt[l], q.get(l));
    sx = tree_sum(sx, red);
    sy = tree_sum(sy, red);
    if (threadIdx.x == 0) {
      uint64_t* rec = d.partial + local * kEpWords;
      rec[0] = __double_as_longlong(sx);
      rec[1] = __double_as_longlong(sy);
#pragma unroll
      for (int l = 0; l < 10; ++l) rec[2 + l] = cnt[l];
    }
    __syncthreads();  // cnt and red reused by the next unit
  }
}

__global__ __launch_bounds__(kEpThreads) void ep_reduce_kernel(EpGroup g) {
  __shared__ double red[kEpThreads];
  __shared__ unsigned long long cnt[10];
  const EpDesc& d = g.d[blockIdx.x];
  double sx = 0.0, sy = 0.0;
  uint64_t q[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (threadIdx.x < 10) cnt[threadIdx.x] = 0;
  for (uint64_t i = threadIdx.x; i < d.units; i += kEpThreads) {
    const uint64_t* rec = d.partial + i * kEpWords;
    sx += __longlong_as_double(rec[0]);
    sy += __longlong_as_double(rec[1]);
#pragma unroll
    for (int l = 0; l < 10; ++l) q[l] += rec[2 + l];
  }
  __syncthreads();
#pragma unroll
  for (int l = 0; l < 10; ++l)
    if (q[l]) atomicAdd(&cnt[l], static_cast<unsigned long long>(q[l]));
  sx = tree_sum(sx, red);
  sy = tree_sum(sy, red);
  if (threadIdx.x == 0) {
    d.out[0] = __double_as_longlong(sx);
    d.out[1] = __double_as_longlong(sy);
#pragma unroll
    for (int l = 0; l < 10; ++l) d.out[2 + l] = cnt[l];
  }
}

}  // namespace

void finalize_ep_group(EpGroup& g) {
  uint64_t u = 0;
  for (uint32_t i = 0; i < g.count; ++i) {
    g.d[i].unit_begin = u;
    g.d[i].units = (g.d[i].n + kEpUnit - 1) / kEpUnit;
    u += g.d[i].units;
  }
  g.total_units = u;
}

hipError_t launch_ep_group(const EpGroup& g, hipStream_t s, int grid_cap) {
  const int cap = grid_cap > 0 ? grid_cap : kEpGrid;
  const int grid = static_cast<int>(std::min<uint64_t>(g.total_units, static_cast<uint64_t>(cap)));
  const hipError_t e = launch_group(ep_units_kernel, grid, kEpThreads, s, g);
  if (e != hipSuccess) return e;
  return launch_group(ep_reduce_kernel, static_cast<int>(g.count), kEpThreads, s, g);
}

}  // namespace gvm
