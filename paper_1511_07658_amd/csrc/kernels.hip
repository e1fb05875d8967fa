// Per-rank kernels of the GVM, written for gfx950 (CDNA4, wave64).
//
//  * vector add / multiply (Table 3 "VecAdd", "VecMul"): streaming, HBM-bound;
//  * Black-Scholes call + put (Table 3 "BlackScholes"): streaming, HBM-bound
//    with a transcendental-heavy body;
//  * SGEMM C = A B (Table 3 "MM", single precision): FP32 MFMA
//    (v_mfma_f32_32x32x2_f32) on LDS-staged, double-buffered tiles.
//
// All three are *grouped persistent* launches: one grid walks the work units
// (vector chunks or GEMM tiles) of every request of the group.  The unit ->
// request map is a search over the per-request first unit, held in the kernel
// arguments.  A unit is always computed by the same code in the same order,
// whatever else is in the group, so a rank's output is bit-identical alone
// and in the mix.
#include "kernels.hpp"

#include <algorithm>
#include <cstdlib>

namespace gvm {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;   // MI355X: workgroup w is dispatched to XCD w % 8

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <class G>
__device__ __forceinline__ int find_request(const G& g, uint64_t u) {
  int lo = 0, hi = static_cast<int>(g.count) - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (g.d[mid].unit_begin <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- vectors

struct AddOp { __device__ __forceinline__ float operator()(float x, float y) const { return x + y; } };
struct MulOp { __device__ __forceinline__ float operator()(float x, float y) const { return x * y; } };

template <class Op>
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
        va[j] = __builtin_nontemporal_load(a4 + threadIdx.x + j * kThreads);
        vb[j] = __builtin_nontemporal_load(b4 + threadIdx.x + j * kThreads);
      }
#pragma unroll
      for (int j = 0; j < kV4; ++j) {
        f32x4 c;
        c.x = op(va[j].x, vb[j].x);
        c.y = op(va[j].y, vb[j].y);
        c.z = op(va[j].z, vb[j].z);
        c.w = op(va[j].w, vb[j].w);
        __builtin_nontemporal_store(c, c4 + threadIdx.x + j * kThreads);
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

__global__ __launch_bounds__(kThreads) void bs_group_kernel(BsGroup g) {
  constexpr int kV4 = kBsUnit / 4 / kThreads;
  const float r = g.rate, v = g.volatility, half_v2 = 0.5f * g.volatility * g.volatility;
  for (uint64_t u = blockIdx.x; u < g.total_units; u += gridDim.x) {
    const int q = find_request(g, u);
    const BsDesc& d = g.d[q];
    const uint64_t e0 = (u - d.unit_begin) * kBsUnit;
    const uint64_t e1 = min(e0 + kBsUnit, d.n);
    const bool aligned = ((reinterpret_cast<uintptr_t>(d.S) | reinterpret_cast<uintptr_t>(d.K) |
                           reinterpret_cast<uintptr_t>(d.T) | reinterpret_cast<uintptr_t>(d.call) |
                           reinterpret_cast<uintptr_t>(d.put)) & 15) == 0;
    if (aligned && e1 - e0 == kBsUnit) {
      const f32x4* S4 = reinterpret_cast<const f32x4*>(d.S + e0);
      const f32x4* K4 = reinterpret_cast<const f32x4*>(d.K + e0);
      const f32x4* T4 = reinterpret_cast<const f32x4*>(d.T + e0);
      f32x4* C4 = reinterpret_cast<f32x4*>(d.call + e0);
      f32x4* P4 = reinterpret_cast<f32x4*>(d.put + e0);
      f32x4 s[kV4], k[kV4], t[kV4];
#pragma unroll
      for (int j = 0; j < kV4; ++j) {
        s[j] = __builtin_nontemporal_load(S4 + threadIdx.x + j * kThreads);
        k[j] = __builtin_nontemporal_load(K4 + threadIdx.x + j * kThreads);
        t[j] = __builtin_nontemporal_load(T4 + threadIdx.x + j * kThreads);
      }
#pragma unroll
      for (int j = 0; j < kV4; ++j) {
        float c0, c1, c2, c3, p0, p1, p2, p3;
        bs_price(s[j].x, k[j].x, t[j].x, r, v, half_v2, c0, p0);
        bs_price(s[j].y, k[j].y, t[j].y, r, v, half_v2, c1, p1);
        bs_price(s[j].z, k[j].z, t[j].z, r, v, half_v2, c2, p2);
        bs_price(s[j].w, k[j].w, t[j].w, r, v, half_v2, c3, p3);
        const f32x4 c = {c0, c1, c2, c3};
        const f32x4 p = {p0, p1, p2, p3};
        __builtin_nontemporal_store(c, C4 + threadIdx.x + j * kThreads);
        __builtin_nontemporal_store(p, P4 + threadIdx.x + j * kThreads);
      }
    } else {
      for (uint64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
        float c, p;
        bs_price(d.S[e], d.K[e], d.T[e], r, v, half_v2, c, p);
        d.call[e] = c;
        d.put[e] = p;
      }
    }
  }
}

// ---------------------------------------------------------------- SGEMM
//
// Workgroup tile BM x BN, k-step BK, WM x WN waves; each wave owns a
// (BM/WM) x (BN/WN) block of C as (BM/WM/32) x (BN/WN/32) accumulators of
// one 32x32 MFMA each.  v_mfma_f32_32x32x2_f32 multiplies a 32x2 slice of A
// by a 2x32 slice of B; lane l supplies A[l%32][k(l)] and B[k(l)][l%32] and
// lane group g = l/32 selects which of the two k values it carries.  Within
// a BK tile, MFMA step s takes k = s for g = 0 and k = BK/2 + s for g = 1, so
// that one lane's A values for the whole tile are contiguous in LDS
// (vector reads).  A is staged row-major, B row-major, both with 4 floats of
// row padding; the next tile is fetched into registers while the current one
// is multiplied, then written to the other LDS buffer (one barrier per tile).
//
// Persistent grid, XCD-aware: the units (tiles, requests in order, tiles of a
// request row-major) are dealt to the 8 XCDs in contiguous blocks, so that
// tiles sharing rows of A and columns of B share an L2.

template <int BM, int BN, int BK, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void sgemm_group_kernel(GemmGroup g) {
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KH = BK / 2;
  constexpr int AST = BK + 4;
  constexpr int BST = BN + 4;
  constexpr int A4 = BM * BK / 4 / NT;   // float4 of A per thread per tile
  constexpr int B4 = BK * BN / 4 / NT;   // float4 of B per thread per tile
  static_assert(TM % 32 == 0 && TN % 32 == 0, "wave tile must be a multiple of 32");
  static_assert(KH % 4 == 0, "BK must be a multiple of 8");
  static_assert(A4 >= 1 && B4 >= 1 && A4 * NT * 4 == BM * BK && B4 * NT * 4 == BK * BN, "tile/threads mismatch");

  __shared__ __attribute__((aligned(16))) float As[2][BM * AST];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK * BST];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 31, lg = lane >> 5;

  // XCD-aware order: with G a multiple of 8, workgroup w runs on XCD w % 8;
  // renumbering it v = (w % 8) * (G / 8) + w / 8 gives each XCD a contiguous
  // block of units in every round of the stride loop below.
  const uint32_t G = gridDim.x;
  const uint32_t U = g.total_units;
  uint32_t v = blockIdx.x;
  if (G % kXcds == 0) v = (blockIdx.x % kXcds) * (G / kXcds) + blockIdx.x / kXcds;

  for (uint32_t u = v; u < U; u += G) {
    const int q = find_request(g, u);
    const GemmDesc& d = g.d[q];
    const int n = static_cast<int>(d.n);
    const uint32_t local = u - d.unit_begin;
    const int row0 = static_cast<int>(local / d.tiles_n) * BM;
    const int col0 = static_cast<int>(local % d.tiles_n) * BN;
    const float* __restrict__ A = d.A;
    const float* __restrict__ B = d.B;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{0};

    f32x4 ra[A4], rb[B4];
    auto load_tile = [&](int k0) {
#pragma unroll
      for (int i = 0; i < A4; ++i) {
        const int f = tid + i * NT;
        const int r = f / (BK / 4), c = (f % (BK / 4)) * 4;
        const int gr = row0 + r, gc = k0 + c;
        if (VEC) {
          ra[i] = (gr < n && gc < n) ? *reinterpret_cast<const f32x4*>(A + static_cast<size_t>(gr) * n + gc)
                                     : f32x4{0};
        } else {
          f32x4 v;
          v.x = (gr < n && gc + 0 < n) ? A[static_cast<size_t>(gr) * n + gc + 0] : 0.0f;
          v.y = (gr < n && gc + 1 < n) ? A[static_cast<size_t>(gr) * n + gc + 1] : 0.0f;
          v.z = (gr < n && gc + 2 < n) ? A[static_cast<size_t>(gr) * n + gc + 2] : 0.0f;
          v.w = (gr < n && gc + 3 < n) ? A[static_cast<size_t>(gr) * n + gc + 3] : 0.0f;
          ra[i] = v;
        }
      }
#pragma unroll
      for (int i = 0; i < B4; ++i) {
        const int f = tid + i * NT;
        const int r = f / (BN / 4), c = (f % (BN / 4)) * 4;
        const int gr = k0 + r, gc = col0 + c;
        if (VEC) {
          rb[i] = (gr < n && gc < n) ? *reinterpret_cast<const f32x4*>(B + static_cast<size_t>(gr) * n + gc)
                                     : f32x4{0};
        } else {
          f32x4 v;
          v.x = (gr < n && gc + 0 < n) ? B[static_cast<size_t>(gr) * n + gc + 0] : 0.0f;
          v.y = (gr < n && gc + 1 < n) ? B[static_cast<size_t>(gr) * n + gc + 1] : 0.0f;
          v.z = (gr < n && gc + 2 < n) ? B[static_cast<size_t>(gr) * n + gc + 2] : 0.0f;
          v.w = (gr < n && gc + 3 < n) ? B[static_cast<size_t>(gr) * n + gc + 3] : 0.0f;
          rb[i] = v;
        }
      }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
      for (int i = 0; i < A4; ++i) {
        const int f = tid + i * NT;
        const int r = f / (BK / 4), c = (f % (BK / 4)) * 4;
        *reinterpret_cast<f32x4*>(&As[buf][r * AST + c]) = ra[i];
      }
#pragma unroll
      for (int i = 0; i < B4; ++i) {
        const int f = tid + i * NT;
        const int r = f / (BN / 4), c = (f % (BN / 4)) * 4;
        *reinterpret_cast<f32x4*>(&Bs[buf][r * BST + c]) = rb[i];
      }
    };

    const int ktiles = (n + BK - 1) / BK;
    load_tile(0);
    store_tile(0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < ktiles) load_tile((kt + 1) * BK);
      float af[FM][KH];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const float* src = &As[buf][(wm * TM + i * 32 + li) * AST + lg * KH];
#pragma unroll
        for (int j = 0; j < KH; j += 4) {
          const f32x4 v = *reinterpret_cast<const f32x4*>(src + j);
          af[i][j] = v.x; af[i][j + 1] = v.y; af[i][j + 2] = v.z; af[i][j + 3] = v.w;
        }
      }
#pragma unroll
      for (int s = 0; s < KH; ++s) {
        float bf[FN];
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[j] = Bs[buf][(lg * KH + s) * BST + wn * TN + j * 32 + li];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][s], bf[j], acc[i][j], 0, 0, 0);
      }
      if (kt + 1 < ktiles) store_tile(buf ^ 1);
      __syncthreads();
    }

    float* __restrict__ C = d.C;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int col = col0 + wn * TN + j * 32 + li;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + wm * TM + i * 32 + 8 * (r / 4) + 4 * lg + (r % 4);
          if (row < n && col < n) C[static_cast<size_t>(row) * n + col] = acc[i][j][r];
        }
      }
  }
}

// Tile configurations.  Index order is part of the tuner table format.
const GemmConfig kGemmConfigs[] = {
    {0, 64, 64, 16, 2, 2},
    {1, 128, 64, 16, 2, 2},
    {2, 128, 128, 16, 2, 2},
    {3, 128, 128, 32, 2, 2},
    {4, 256, 128, 16, 4, 2},
    {5, 128, 256, 16, 2, 4},
    {6, 256, 128, 32, 4, 2},
    {7, 64, 128, 16, 2, 2},
};
constexpr int kNumGemmConfigs = sizeof(kGemmConfigs) / sizeof(kGemmConfigs[0]);

int g_forced_config = -1;

#include "gemm_tiles.inc"   // kTileTable: (n_max, config index) rows written by the tuner

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_cfg(const GemmGroup& g, bool vec, hipStream_t s, int grid_cap) {
  constexpr int NT = WM * WN * 64;
  int cap = grid_cap > 0 ? grid_cap : 256 * 2;
  int grid = static_cast<int>(std::min<uint32_t>(g.total_units, static_cast<uint32_t>(cap)));
  if (grid <= 0) return hipSuccess;
  if (grid > kXcds) grid -= grid % kXcds;  // whole rounds over the 8 XCDs
  if (vec)
    hipLaunchKernelGGL((sgemm_group_kernel<BM, BN, BK, WM, WN, true>), dim3(grid), dim3(NT), 0, s, g);
  else
    hipLaunchKernelGGL((sgemm_group_kernel<BM, BN, BK, WM, WN, false>), dim3(grid), dim3(NT), 0, s, g);
  return hipGetLastError();
}

}  // namespace

int gemm_config_count() { return kNumGemmConfigs; }
const GemmConfig& gemm_config(int idx) { return kGemmConfigs[idx]; }
void gemm_config_force(int idx) { g_forced_config = (idx >= 0 && idx < kNumGemmConfigs) ? idx : -1; }

int gemm_config_for(uint64_t n) {
  if (g_forced_config >= 0) return g_forced_config;
  // tuning and tests only: force one configuration for every size
  if (const char* env = getenv("GVM_SGEMM_CONFIG")) {
    const int c = atoi(env);
    if (c >= 0 && c < kNumGemmConfigs) return c;
  }
  for (const auto& row : kTileTable)
    if (n <= row[0]) return static_cast<int>(row[1]);
  return kTileTable[sizeof(kTileTable) / sizeof(kTileTable[0]) - 1][1];
}

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

void finalize_gemm_group(GemmGroup& g, int config_idx) {
  const GemmConfig& c = kGemmConfigs[config_idx];
  uint32_t u = 0;
  for (uint32_t i = 0; i < g.count; ++i) {
    const uint32_t n = g.d[i].n;
    const uint32_t tm = (n + c.bm - 1) / c.bm, tn = (n + c.bn - 1) / c.bn;
    g.d[i].tiles_n = tn;
    g.d[i].unit_begin = u;
    g.d[i].units = tm * tn;
    u += tm * tn;
  }
  g.total_units = u;
}

hipError_t launch_vecadd_group(const VecGroup& g, hipStream_t s, int grid_cap) {
  int cap = grid_cap > 0 ? grid_cap : 1024;
  int grid = static_cast<int>(std::min<uint64_t>(g.total_units, static_cast<uint64_t>(cap)));
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(vec_group_kernel<AddOp>, dim3(grid), dim3(kThreads), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_vecmul_group(const VecGroup& g, hipStream_t s, int grid_cap) {
  int cap = grid_cap > 0 ? grid_cap : 1024;
  int grid = static_cast<int>(std::min<uint64_t>(g.total_units, static_cast<uint64_t>(cap)));
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(vec_group_kernel<MulOp>, dim3(grid), dim3(kThreads), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_bs_group(const BsGroup& g, hipStream_t s, int grid_cap) {
  int cap = grid_cap > 0 ? grid_cap : 1024;
  int grid = static_cast<int>(std::min<uint64_t>(g.total_units, static_cast<uint64_t>(cap)));
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(bs_group_kernel, dim3(grid), dim3(kThreads), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_sgemm_group(const GemmGroup& g, int config_idx, hipStream_t s, int grid_cap) {
  bool vec = true;
  for (uint32_t i = 0; i < g.count; ++i)
    if ((g.d[i].n % 4) != 0 || (reinterpret_cast<uintptr_t>(g.d[i].A) & 15) ||
        (reinterpret_cast<uintptr_t>(g.d[i].B) & 15))
      vec = false;
  switch (config_idx) {
    case 0: return launch_cfg<64, 64, 16, 2, 2>(g, vec, s, grid_cap);
    case 1: return launch_cfg<128, 64, 16, 2, 2>(g, vec, s, grid_cap);
    case 2: return launch_cfg<128, 128, 16, 2, 2>(g, vec, s, grid_cap);
    case 3: return launch_cfg<128, 128, 32, 2, 2>(g, vec, s, grid_cap);
    case 4: return launch_cfg<256, 128, 16, 4, 2>(g, vec, s, grid_cap);
    case 5: return launch_cfg<128, 256, 16, 2, 4>(g, vec, s, grid_cap);
    case 6: return launch_cfg<256, 128, 32, 4, 2>(g, vec, s, grid_cap);
    case 7: return launch_cfg<64, 128, 16, 2, 2>(g, vec, s, grid_cap);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gvm
