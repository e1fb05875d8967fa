// Streaming per-rank kernels of the GVM, written for gfx950 (CDNA4, wave64):
//
//  * vector add / multiply (Table 3 "VecAdd", "VecMul"): HBM-bound;
//  * Black-Scholes call + put (Table 3 "BlackScholes"): HBM-bound with a
//    transcendental-heavy body.
//
// Both are grouped persistent launches: one grid walks the work units (vector
// chunks) of every request of the group; the unit -> request map is a search
// over the per-request first unit held in the kernel arguments.  A unit is
// always computed by the same code in the same order, whatever else is in the
// group, so a rank's output is bit-identical alone and in the mix.
#include "group_device.hpp"

#include <algorithm>
#include <cstdlib>

namespace gvm {

namespace {

// Launch shapes measured on the MI355X (sweeps of grid, float4 per thread
// and cache policy over the grouped launches): one workgroup per work unit
// beats every persistent grid (512 to 4096 workgroups) for groups beyond the
// memory-side cache, since the dispatcher keeps every SIMD at its register-
// limited occupancy and balances the tail; for small groups the two
// coincide.  A group whose bytes exceed the 256 MB memory-side cache
// streams through with non-temporal loads and stores; a smaller one stays
// cacheable, since its inputs come back from that cache on the next request.
constexpr int kVecGrid = 1 << 24;     // i.e. one workgroup per unit
constexpr int kBsGrid = 1 << 24;
constexpr int kBsV4 = 4;              // float4 per thread per stream of a Black-Scholes unit
constexpr uint64_t kMallBytes = 256ull << 20;

// ---------------------------------------------------------------- vectors

struct AddOp { __device__ __forceinline__ float operator()(float x, float y) const { return x + y; } };
struct MulOp { __device__ __forceinline__ float operator()(float x, float y) const { return x * y; } };

template <class T, bool NT>
__device__ __forceinline__ T stream_load(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <class T, bool NT>
__device__ __forceinline__ void stream_store(T v, T* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <class Op, bool NT>
__global__ __launch_bounds__(kThreads) void vec_group_kernel(VecGroup g) {
  constexpr int kV4 = kVecUnit / 4 / kThreads;  // float4 per thread per unit
  Op op;
  for (uint64_t u = blockIdx.x; u < g.total_units; u += gridDim.x) {
    const int r = find_request(g, u);
    const VecDesc& d = g.d[r];
    const uint64_t e0 = (u - d.unit_begin) * kVecUnit;
    const uint64_t e1 = min(e0 + kVecUnit, d.n);
    const bool aligned = ((reinterpret_cast<uintptr_t>(d.a) | reinterpret_cast<uintptr_t>(d.b) |
                           reinterpret_cast<uintptr_t>(d.c)) & 15) == 0;
    if (aligned && e1 - e0 == kVecUnit) {
      const f32x4* a4 = reinterpret_cast<const f32x4*>(d.a + e0);
      const f32x4* b4 = reinterpret_cast<const f32x4*>(d.b + e0);
      f32x4* c4 = reinterpret_cast<f32x4*>(d.c + e0);
      f32x4 va[kV4], vb[kV4];
#pragma unroll
      for (int j = 0; j < kV4; ++j) {
        va[j] = stream_load<f32x4, NT>(a4 + threadIdx.x + j * kThreads);
        vb[j] = stream_load<f32x4, NT>(b4 + threadIdx.x + j * kThreads);
      }
#pragma unroll
      for (int j = 0; j < kV4; ++j) {
        f32x4 c;
        c.x = op(va[j].x, vb[j].x);
        c.y = op(va[j].y, vb[j].y);
        c.z = op(va[j].z, vb[j].z);
        c.w = op(va[j].w, vb[j].w);
        stream_store<f32x4, NT>(c, c4 + threadIdx.x + j * kThreads);
      }
    } else {
      for (uint64_t e = e0 + threadIdx.x; e < e1; e += kThreads) d.c[e] = op(d.a[e], d.b[e]);
    }
  }
}

// ---------------------------------------------------------------- Black-Scholes
//
// Standard normal distribution function from the polynomial approximation of
// Abramowitz and Stegun, Handbook of Mathematical Functions, formula 26.2.17
// (absolute error below 7.5e-8):
//   N(x) = 1 - phi(x) (b1 t + b2 t^2 + b3 t^3 + b4 t^4 + b5 t^5),  t = 1/(1 + p x),  x >= 0
// and N(x) = 1 - N(-x) for x < 0.  The pricing formula itself is the
// Black-Scholes (1973) one of the reference:
//   d1 = (ln(S/K) + (r + sigma^2/2) T) / (sigma sqrt T),  d2 = d1 - sigma sqrt T
//   call = S N(d1) - K e^{-rT} N(d2),  put = K e^{-rT} (1 - N(d2)) - S (1 - N(d1))

__device__ __forceinline__ float norm_cdf_as(float x) {
  constexpr float p = 0.2316419f;
  constexpr float b1 = 0.319381530f, b2 = -0.356563782f, b3 = 1.781477937f, b4 = -1.821255978f,
                  b5 = 1.330274429f;
  constexpr float inv_sqrt_2pi = 0.39894228040143267794f;
  const float ax = fabsf(x);
  const float t = __frcp_rn(fmaf(p, ax, 1.0f));
  const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, b5, b4), b3), b2), b1);
  const float phi = inv_sqrt_2pi * __expf(-0.5f * ax * ax);
  const float upper = phi * poly;          // 1 - N(|x|)
  return x >= 0.0f ? 1.0f - upper : upper;
}

__device__ __forceinline__ void bs_price(float S, float K, float T, float r, float v, float half_v2,
                                         float& call, float& put) {
  const float rs = __frsqrt_rn(T);
  const float sqrt_t = T * rs;
  const float vs = v * sqrt_t;
  const float d1 = (__logf(__fdividef(S, K)) + (r + half_v2) * T) * __fdividef(rs, v);
  const float d2 = d1 - vs;
  const float kd = K * __expf(-r * T);
  const float n1 = norm_cdf_as(d1);
  const float n2 = norm_cdf_as(d2);
  call = S * n1 - kd * n2;
  put = kd * (1.0f - n2) - S * (1.0f - n1);
}

// Registers of one work unit: V4 float4 per thread of each input stream
// (V4 * 1024 options per unit of 256 threads).
template <int V4>
struct BsUnitRegs {
  f32x4 s[V4], k[V4], t[V4];
};

// Locate unit u and, when it is full and its streams are 16-byte aligned,
// issue its loads; a ragged or unaligned unit returns false and is left to
// the element-wise path.
template <int V4, bool NT>
__device__ __forceinline__ bool bs_load(const BsGroup& g, uint64_t u, int& q, uint64_t& e0, BsUnitRegs<V4>& x) {
  constexpr uint64_t kUnit = V4 * 4 * kThreads;
  q = find_request(g, u);
  const BsDesc& d = g.d[q];
  e0 = (u - d.unit_begin) * kUnit;
  const uint64_t e1 = min(e0 + kUnit, d.n);
  const bool aligned = ((reinterpret_cast<uintptr_t>(d.S) | reinterpret_cast<uintptr_t>(d.K) |
                         reinterpret_cast<uintptr_t>(d.T) | reinterpret_cast<uintptr_t>(d.call) |
                         reinterpret_cast<uintptr_t>(d.put)) & 15) == 0;
  if (!aligned || e1 - e0 != kUnit) return false;
  const f32x4* S4 = reinterpret_cast<const f32x4*>(d.S + e0);
  const f32x4* K4 = reinterpret_cast<const f32x4*>(d.K + e0);
  const f32x4* T4 = reinterpret_cast<const f32x4*>(d.T + e0);
#pragma unroll
  for (int j = 0; j < V4; ++j) {
    x.s[j] = stream_load<f32x4, NT>(S4 + threadIdx.x + j * kThreads);
    x.k[j] = stream_load<f32x4, NT>(K4 + threadIdx.x + j * kThreads);
    x.t[j] = stream_load<f32x4, NT>(T4 + threadIdx.x + j * kThreads);
  }
  return true;
}

template <int V4, bool NT>
__device__ __forceinline__ void bs_price_store(const BsDesc& d, uint64_t e0, const BsUnitRegs<V4>& x, float r,
                                               float v, float half_v2) {
  f32x4* C4 = reinterpret_cast<f32x4*>(d.call + e0);
  f32x4* P4 = reinterpret_cast<f32x4*>(d.put + e0);
#pragma unroll
  for (int j = 0; j < V4; ++j) {
    float c0, c1, c2, c3, p0, p1, p2, p3;
    bs_price(x.s[j].x, x.k[j].x, x.t[j].x, r, v, half_v2, c0, p0);
    bs_price(x.s[j].y, x.k[j].y, x.t[j].y, r, v, half_v2, c1, p1);
    bs_price(x.s[j].z, x.k[j].z, x.t[j].z, r, v, half_v2, c2, p2);
    bs_price(x.s[j].w, x.k[j].w, x.t[j].w, r, v, half_v2, c3, p3);
    const f32x4 c = {c0, c1, c2, c3};
    const f32x4 p = {p0, p1, p2, p3};
    stream_store<f32x4, NT>(c, C4 + threadIdx.x + j * kThreads);
    stream_store<f32x4, NT>(p, P4 + threadIdx.x + j * kThreads);
  }
}

// Ragged or unaligned unit: one option per thread and step.
template <int V4>
__device__ __forceinline__ void bs_unit_elementwise(const BsDesc& d, uint64_t e0, float r, float v, float half_v2) {
  constexpr uint64_t kUnit = V4 * 4 * kThreads;
  const uint64_t e1 = min(e0 + kUnit, d.n);
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
    float c, p;
    bs_price(d.S[e], d.K[e], d.T[e], r, v, half_v2, c, p);
    d.call[e] = c;
    d.put[e] = p;
  }
}

// V4: float4 per thread of each stream per unit.  Every option is priced by
// the same code whatever the shape or the group.
template <int V4, bool NT>
__global__ __launch_bounds__(kThreads) void bs_group_kernel(BsGroup g) {
  const float r = g.rate, v = g.volatility, half_v2 = 0.5f * g.volatility * g.volatility;
  for (uint64_t u = blockIdx.x; u < g.total_units; u += gridDim.x) {
    int q;
    uint64_t e0;
    BsUnitRegs<V4> x;
    if (bs_load<V4, NT>(g, u, q, e0, x)) bs_price_store<V4, NT>(g.d[q], e0, x, r, v, half_v2);
    else bs_unit_elementwise<V4>(g.d[q], e0, r, v, half_v2);
  }
}

}  // namespace

void finalize_vec_group(VecGroup& g) {
  uint64_t u = 0;
  for (uint32_t i = 0; i < g.count; ++i) {
    g.d[i].unit_begin = u;
    u += (g.d[i].n + kVecUnit - 1) / kVecUnit;
  }
  g.total_units = u;
}

void finalize_bs_group(BsGroup& g) {
  uint64_t u = 0;
  for (uint32_t i = 0; i < g.count; ++i) {
    g.d[i].unit_begin = u;
    u += (g.d[i].n + kBsUnit - 1) / kBsUnit;
  }
  g.total_units = u;
}

// Tuning overrides (read once per process): GVM_STREAM_GRID replaces the
// grid, GVM_STREAM_NT = 0 / 1 forces cached / non-temporal access.
int stream_grid(int grid_cap, int dflt) {
  static const int env = [] {
    const char* e = getenv("GVM_STREAM_GRID");
    return e ? atoi(e) : 0;
  }();
  if (grid_cap > 0) return grid_cap;
  return env > 0 ? env : dflt;
}

bool stream_nt(uint64_t group_bytes) {
  static const int env = [] {
    const char* e = getenv("GVM_STREAM_NT");
    return e ? atoi(e) : -1;
  }();
  return env >= 0 ? env != 0 : group_bytes > kMallBytes;
}

template <class Op>
hipError_t launch_vec(const VecGroup& g, hipStream_t s, int grid_cap) {
  const int grid = static_cast<int>(std::min<uint64_t>(g.total_units, static_cast<uint64_t>(stream_grid(grid_cap, kVecGrid))));
  const uint64_t bytes = g.total_units * kVecUnit * 12;
  return stream_nt(bytes) ? launch_group(vec_group_kernel<Op, true>, grid, kThreads, s, g)
                          : launch_group(vec_group_kernel<Op, false>, grid, kThreads, s, g);
}

hipError_t launch_vecadd_group(const VecGroup& g, hipStream_t s, int grid_cap) { return launch_vec<AddOp>(g, s, grid_cap); }

hipError_t launch_vecmul_group(const VecGroup& g, hipStream_t s, int grid_cap) { return launch_vec<MulOp>(g, s, grid_cap); }

// Black-Scholes launch shape: float4 per thread per stream (GVM_BS_V4 = 2, 4
// or 8), read once per process.
int bs_v4() {
  static const int v4 = [] {
    const char* e = getenv("GVM_BS_V4");
    const int x = e ? atoi(e) : kBsV4;
    return (x == 2 || x == 8) ? x : 4;
  }();
  return v4;
}

template <int V4>
hipError_t launch_bs_shape(const BsGroup& g0, hipStream_t s, int grid_cap) {
  // the unit size of the shape: recount the units of a copy of the group
  BsGroup g = g0;
  constexpr uint64_t kUnit = V4 * 4 * kThreads;
  uint64_t u = 0;
  for (uint32_t i = 0; i < g.count; ++i) {
    g.d[i].unit_begin = u;
    u += (g.d[i].n + kUnit - 1) / kUnit;
  }
  g.total_units = u;
  const int grid = static_cast<int>(std::min<uint64_t>(g.total_units, static_cast<uint64_t>(stream_grid(grid_cap, kBsGrid))));
  return stream_nt(g.total_units * kUnit * 20) ? launch_group(bs_group_kernel<V4, true>, grid, kThreads, s, g)
                                               : launch_group(bs_group_kernel<V4, false>, grid, kThreads, s, g);
}

hipError_t launch_bs_group(const BsGroup& g, hipStream_t s, int grid_cap) {
  switch (bs_v4()) {
    case 2: return launch_bs_shape<2>(g, s, grid_cap);
    case 8: return launch_bs_shape<8>(g, s, grid_cap);
    default: return launch_bs_shape<4>(g, s, grid_cap);
  }
}

}  // namespace gvm
