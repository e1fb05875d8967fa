// Device ceilings of the MI355X the GVM runs on:
//   copy   <MiB> <reps>   plain device-to-device copy kernel (HBM read+write rate;
//                         also the reference kernel for scaling FETCH_SIZE/WRITE_SIZE)
//   stream <M floats>     the Black-Scholes access mix (three input streams, two
//                         output streams) and its read-only and write-only halves,
//                         over float4s per thread, grid and cache policy
//   mfma   <iters>        FP32 MFMA issue rate (v_mfma_f32_32x32x2_f32 chains)
//   pcie   <MiB>          pinned host<->device copy rates, one direction and both
//   link   <MiB> [piece]  the manager's transfer path alone: 8 MiB (or [piece] MiB) pieces to and from
//                         non-coherent pinned memory, each way, both, and the 2:1 mix
//   hostcopy <MiB>        CPU memcpy pageable <-> pinned, 1 and 8 threads
//   latency <iters>       launch -> completion seen by the host (event query,
//                         stream synchronize, kernel-written host flag)
//   init                  time to create the device context in a fresh process
// Prints one JSON object per test.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#define CK(x)                                                                          \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));                   \
      exit(2);                                                                         \
    }                                                                                  \
  } while (0)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void copy_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst, size_t n4) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n4; i += static_cast<size_t>(gridDim.x) * 256ull)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Streaming variants: plain (cached) loads/stores, U float4 per thread per round.
template <int U, bool NT>
__global__ __launch_bounds__(256) void copy_var_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst, size_t n4) {
  const size_t stride = static_cast<size_t>(gridDim.x) * 256ull * U;
  for (size_t base = blockIdx.x * 256ull * U + threadIdx.x; base < n4; base += stride) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + u * 256ull;
      if (i < n4) v[u] = NT ? __builtin_nontemporal_load(src + i) : src[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + u * 256ull;
      if (i < n4) {
        if (NT) __builtin_nontemporal_store(v[u], dst + i); else dst[i] = v[u];
      }
    }
  }
}

template <bool NT>
__device__ __forceinline__ f32x4 ld4(const f32x4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT>
__device__ __forceinline__ void st4(f32x4 v, f32x4* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Three streams in, two out (o1 = a + b, o2 = b + c): Black-Scholes' 12 B
// read and 8 B written per element without its arithmetic.  U float4 per
// thread per round, grid-stride.
template <int U, bool NT>
__global__ __launch_bounds__(256) void mix32_kernel(const f32x4* __restrict__ a, const f32x4* __restrict__ b,
                                                    const f32x4* __restrict__ c, f32x4* __restrict__ o1,
                                                    f32x4* __restrict__ o2, size_t n4) {
  const size_t stride = static_cast<size_t>(gridDim.x) * 256ull * U;
  for (size_t base = blockIdx.x * 256ull * U + threadIdx.x; base < n4; base += stride) {
    f32x4 va[U], vb[U], vc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + u * 256ull;
      if (i < n4) {
        va[u] = ld4<NT>(a + i);
        vb[u] = ld4<NT>(b + i);
        vc[u] = ld4<NT>(c + i);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + u * 256ull;
      if (i < n4) {
        st4<NT>(va[u] + vb[u], o1 + i);
        st4<NT>(vb[u] + vc[u], o2 + i);
      }
    }
  }
}

// Read half: three streams summed per thread, one float per thread written.
template <int U, bool NT>
__global__ __launch_bounds__(256) void read3_kernel(const f32x4* __restrict__ a, const f32x4* __restrict__ b,
                                                    const f32x4* __restrict__ c, float* __restrict__ sink, size_t n4) {
  const size_t stride = static_cast<size_t>(gridDim.x) * 256ull * U;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (size_t base = blockIdx.x * 256ull * U + threadIdx.x; base < n4; base += stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + u * 256ull;
      if (i < n4) acc += ld4<NT>(a + i) + ld4<NT>(b + i) + ld4<NT>(c + i);
    }
  }
  sink[blockIdx.x * 256ull + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

// Write half: two streams written from the index.
template <int U, bool NT>
__global__ __launch_bounds__(256) void write2_kernel(f32x4* __restrict__ o1, f32x4* __restrict__ o2, size_t n4) {
  const size_t stride = static_cast<size_t>(gridDim.x) * 256ull * U;
  for (size_t base = blockIdx.x * 256ull * U + threadIdx.x; base < n4; base += stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + u * 256ull;
      if (i < n4) {
        const float f = static_cast<float>(i);
        st4<NT>(f32x4{f, f, f, f}, o1 + i);
        st4<NT>(f32x4{f, -f, f, -f}, o2 + i);
      }
    }
  }
}

__global__ __launch_bounds__(256) void mfma_kernel(float* out, int iters) {
  f32x16 a0 = {0}, a1 = {0}, a2 = {0}, a3 = {0};
  const float x = threadIdx.x * 1e-3f, y = 1.0f;
  for (int i = 0; i < iters; ++i) {
    a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a1, 0, 0, 0);
    a2 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a2, 0, 0, 0);
    a3 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a3, 0, 0, 0);
  }
  float s = 0.0f;
  for (int r = 0; r < 16; ++r) s += a0[r] + a1[r] + a2[r] + a3[r];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void empty_kernel(int x) {
  if (x < 0 && threadIdx.x == 0) asm volatile("s_nop 0");
}

// Lane 0 publishes `v` to pinned host memory (global store, system scope).
__global__ void signal_kernel(uint32_t* flag, uint32_t v) {
  if (threadIdx.x == 0) __hip_atomic_store(flag, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

struct Big {
  float v[320];  // 1280 bytes, like a grouped launch's request table
};

__global__ void big_arg_kernel(Big b) {
  if (b.v[0] < 0.0f && threadIdx.x == 0) asm volatile("s_nop 0");
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The mix of the copy-inclusive batches (vector add, SGEMM): twice as many
// bytes in as out, 8 MiB pieces, one stream per direction, an output piece
// queued after every second input piece; best of 3 timed rounds after one
// warm-up (GB/s over both directions).
static double pcie_in2_out1(void* d1, void* h1, void* d2, void* h2, size_t bytes, hipStream_t in, hipStream_t out,
                            size_t piece = size_t(8) << 20) {
  const size_t np = bytes / piece;
  double mix = 0;
  for (int rep = 0; rep < 4; ++rep) {
    const double t0 = now_s();
    for (size_t i = 0; i < np; ++i) {
      CK(hipMemcpyAsync(static_cast<char*>(d1) + i * piece, static_cast<char*>(h1) + i * piece, piece,
                        hipMemcpyHostToDevice, in));
      if (i % 2 == 0)
        CK(hipMemcpyAsync(static_cast<char*>(h2) + (i / 2) * piece, static_cast<char*>(d2) + (i / 2) * piece, piece,
                          hipMemcpyDeviceToHost, out));
    }
    CK(hipStreamSynchronize(in));
    CK(hipStreamSynchronize(out));
    const double moved = static_cast<double>((np + (np + 1) / 2) * piece);
    if (rep > 0) mix = std::max(mix, moved / (now_s() - t0) / 1e9);
  }
  return mix;
}

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: %s copy <MiB> <reps> | mfma <iters> | pcie <MiB> | link <MiB> [piece MiB] | latency <iters> | init\n", argv[0]);
    return 1;
  }
  const std::string what = argv[1];
  if (what == "init") {
    const double t0 = now_s();
    CK(hipSetDevice(0));
    CK(hipFree(nullptr));
    const double t1 = now_s();
    printf("{\"test\":\"init\",\"context_s\":%.6f}\n", t1 - t0);
    return 0;
  }
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  if (strncmp(p.gcnArchName, "gfx950", 6) != 0) {
    fprintf(stderr, "device is %s, not gfx950\n", p.gcnArchName);
    return 2;
  }
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  if (what == "copy") {
    const size_t mib = argc > 2 ? strtoull(argv[2], nullptr, 10) : 2048;
    const int reps = argc > 3 ? atoi(argv[3]) : 10;
    const size_t bytes = mib << 20;
    const size_t n4 = bytes / 16;
    f32x4 *s, *d;
    CK(hipMalloc(&s, bytes));
    CK(hipMalloc(&d, bytes));
    CK(hipMemset(s, 0, bytes));
    const int grid = 256 * 4;
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, nullptr, s, d, n4);
    CK(hipDeviceSynchronize());
    float best = 1e30f, total = 0.0f;
    for (int r = 0; r < reps; ++r) {
      CK(hipEventRecord(e0));
      hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, nullptr, s, d, n4);
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      float ms;
      CK(hipEventElapsedTime(&ms, e0, e1));
      best = ms < best ? ms : best;
      total += ms;
    }
    printf("{\"test\":\"copy\",\"bytes_read\":%zu,\"bytes_written\":%zu,\"launches\":%d,\"avg_ms\":%.6f,"
           "\"best_GBps\":%.1f,\"avg_GBps\":%.1f}\n",
           bytes, bytes, reps + 1, total / reps, 2.0 * bytes / (best * 1e-3) / 1e9,
           2.0 * bytes / (total / reps * 1e-3) / 1e9);
    CK(hipFree(s));
    CK(hipFree(d));
  } else if (what == "copyvar") {
    // HBM streaming variants over a 4 GiB copy (well above the 256 MB MALL)
    const size_t bytes = size_t(argc > 2 ? strtoull(argv[2], nullptr, 10) : 4096) << 20;
    const size_t n4 = bytes / 16;
    f32x4 *src, *dst;
    CK(hipMalloc(&src, bytes));
    CK(hipMalloc(&dst, bytes));
    CK(hipMemset(src, 0, bytes));
    CK(hipMemset(dst, 0, bytes));
    auto timeit = [&](auto launch) {
      launch();
      CK(hipDeviceSynchronize());
      float best = 1e30f;
      for (int r = 0; r < 5; ++r) {
        CK(hipEventRecord(e0));
        launch();
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        float ms;
        CK(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
      }
      return 2.0 * bytes / (best * 1e-3) / 1e9;
    };
    for (int grid : {512, 1024, 2048, 4096, 8192}) {
      const double a = timeit([&] { hipLaunchKernelGGL((copy_var_kernel<1, false>), dim3(grid), dim3(256), 0, nullptr, src, dst, n4); });
      const double b = timeit([&] { hipLaunchKernelGGL((copy_var_kernel<1, true>), dim3(grid), dim3(256), 0, nullptr, src, dst, n4); });
      const double c = timeit([&] { hipLaunchKernelGGL((copy_var_kernel<4, false>), dim3(grid), dim3(256), 0, nullptr, src, dst, n4); });
      const double d = timeit([&] { hipLaunchKernelGGL((copy_var_kernel<4, true>), dim3(grid), dim3(256), 0, nullptr, src, dst, n4); });
      printf("{\"test\":\"copyvar\",\"bytes\":%zu,\"grid\":%d,\"u1_cached_GBps\":%.1f,\"u1_nt_GBps\":%.1f,"
             "\"u4_cached_GBps\":%.1f,\"u4_nt_GBps\":%.1f}\n", bytes, grid, a, b, c, d);
    }
    CK(hipFree(src));
    CK(hipFree(dst));
  } else if (what == "stream") {
    // five arrays of n floats (default 64 M each: 1.34 GB moved by the mix
    // kernel, like sixteen 4M-option Black-Scholes requests)
    const size_t n = size_t(argc > 2 ? strtoull(argv[2], nullptr, 10) : 64) << 20;
    const size_t n4 = n / 4;
    f32x4* buf[5];
    for (auto& b : buf) {
      CK(hipMalloc(&b, n * sizeof(float)));
      CK(hipMemset(b, 0, n * sizeof(float)));
    }
    const int max_grid = static_cast<int>((n4 + 255) / 256);
    float* sink;
    CK(hipMalloc(&sink, static_cast<size_t>(max_grid) * 256 * sizeof(float)));
    auto timeit = [&](auto launch) {
      launch();
      CK(hipDeviceSynchronize());
      float best = 1e30f, total = 0.0f;
      for (int r = 0; r < 5; ++r) {
        CK(hipEventRecord(e0));
        launch();
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        float ms;
        CK(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
        total += ms;
      }
      return std::make_pair(best, total / 5);
    };
    auto report = [&](const char* kind, int u, bool nt, int grid, double bytes, std::pair<float, float> t) {
      printf("{\"test\":\"stream\",\"kind\":\"%s\",\"u\":%d,\"nt\":%d,\"grid\":%d,\"bytes\":%.0f,"
             "\"best_us\":%.2f,\"best_GBps\":%.1f,\"avg_GBps\":%.1f}\n",
             kind, u, nt ? 1 : 0, grid, bytes, t.first * 1e3, bytes / (t.first * 1e-3) / 1e9, bytes / (t.second * 1e-3) / 1e9);
    };
    auto sweep = [&](auto u_tag, auto nt_tag) {
      constexpr int U = decltype(u_tag)::value;
      constexpr bool NT = decltype(nt_tag)::value;
      const int full = static_cast<int>((n4 + 256ull * U - 1) / (256ull * U));
      for (int grid : {256, 512, 1024, 2048, 4096, full}) {
        if (grid > full) continue;
        report("mix3r2w", U, NT, grid, 20.0 * n, timeit([&] {
          hipLaunchKernelGGL((mix32_kernel<U, NT>), dim3(grid), dim3(256), 0, nullptr, buf[0], buf[1], buf[2], buf[3], buf[4], n4);
        }));
        report("read3", U, NT, grid, 12.0 * n, timeit([&] {
          hipLaunchKernelGGL((read3_kernel<U, NT>), dim3(grid), dim3(256), 0, nullptr, buf[0], buf[1], buf[2], sink, n4);
        }));
        report("write2", U, NT, grid, 8.0 * n, timeit([&] {
          hipLaunchKernelGGL((write2_kernel<U, NT>), dim3(grid), dim3(256), 0, nullptr, buf[3], buf[4], n4);
        }));
      }
    };
    using F = std::false_type;
    using T = std::true_type;
    sweep(std::integral_constant<int, 1>{}, F{});
    sweep(std::integral_constant<int, 1>{}, T{});
    sweep(std::integral_constant<int, 2>{}, F{});
    sweep(std::integral_constant<int, 2>{}, T{});
    sweep(std::integral_constant<int, 4>{}, F{});
    sweep(std::integral_constant<int, 4>{}, T{});
    for (auto& b : buf) CK(hipFree(b));
    CK(hipFree(sink));
  } else if (what == "mfma") {
    const int iters = argc > 2 ? atoi(argv[2]) : 20000;
    const int blocks = p.multiProcessorCount * 8;
    float* o;
    CK(hipMalloc(&o, static_cast<size_t>(blocks) * 256 * 4));
    hipLaunchKernelGGL(mfma_kernel, dim3(blocks), dim3(256), 0, nullptr, o, 100);
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    hipLaunchKernelGGL(mfma_kernel, dim3(blocks), dim3(256), 0, nullptr, o, iters);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms;
    CK(hipEventElapsedTime(&ms, e0, e1));
    const double flop = double(blocks) * 4 * iters * 4 * (32.0 * 32 * 2 * 2);
    printf("{\"test\":\"mfma_f32\",\"TFLOPs\":%.2f,\"ms\":%.3f}\n", flop / (ms * 1e-3) / 1e12, ms);
    CK(hipFree(o));
  } else if (what == "pcie") {
    // pinned host <-> device copy rates: warm buffers, 5 repetitions each,
    // for the default and the non-coherent pinned allocation
    const size_t bytes = (argc > 2 ? strtoull(argv[2], nullptr, 10) : 256) << 20;
    const unsigned flag_sets[2] = {hipHostMallocDefault, hipHostMallocNonCoherent};
    const char* names[2] = {"default", "noncoherent"};
    void *d1, *d2;
    CK(hipMalloc(&d1, bytes));
    CK(hipMalloc(&d2, bytes));
    CK(hipMemset(d1, 1, bytes));
    CK(hipMemset(d2, 2, bytes));
    hipStream_t s1, s2;
    CK(hipStreamCreateWithFlags(&s1, hipStreamNonBlocking));
    CK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    for (int f = 0; f < 2; ++f) {
      void *h1, *h2;
      CK(hipHostMalloc(&h1, bytes, flag_sets[f]));
      CK(hipHostMalloc(&h2, bytes, flag_sets[f]));
      memset(h1, 1, bytes);
      memset(h2, 2, bytes);
      double best[3] = {0, 0, 0};
      for (int rep = 0; rep < 6; ++rep) {
        double t0 = now_s();
        CK(hipMemcpyAsync(d1, h1, bytes, hipMemcpyHostToDevice, s1));
        CK(hipStreamSynchronize(s1));
        const double h2d = bytes / (now_s() - t0) / 1e9;
        t0 = now_s();
        CK(hipMemcpyAsync(h2, d2, bytes, hipMemcpyDeviceToHost, s2));
        CK(hipStreamSynchronize(s2));
        const double d2h = bytes / (now_s() - t0) / 1e9;
        t0 = now_s();
        CK(hipMemcpyAsync(d1, h1, bytes, hipMemcpyHostToDevice, s1));
        CK(hipMemcpyAsync(h2, d2, bytes, hipMemcpyDeviceToHost, s2));
        CK(hipStreamSynchronize(s1));
        CK(hipStreamSynchronize(s2));
        const double both = 2.0 * bytes / (now_s() - t0) / 1e9;
        if (rep > 0) {  // the first repetition is a warm-up
          best[0] = std::max(best[0], h2d);
          best[1] = std::max(best[1], d2h);
          best[2] = std::max(best[2], both);
        }
      }
      printf("{\"test\":\"pcie_pinned\",\"alloc\":\"%s\",\"bytes\":%zu,\"h2d_GBps\":%.1f,\"d2h_GBps\":%.1f,\"duplex_GBps\":%.1f}\n",
             names[f], bytes, best[0], best[1], best[2]);
      {
        // the same bytes in pieces of 2 to 16 MiB on one stream per
        // direction, and in 4 MiB pieces dealt round-robin over 2 or 4
        // streams per direction (one direction at a time, then both)
        hipStream_t ps[8];
        for (auto& x : ps) CK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        const std::pair<int, int> shapes[] = {{2, 1}, {4, 1}, {8, 1}, {16, 1}, {4, 2}, {4, 4}};
        for (const auto& sh : shapes) {
          const size_t piece = size_t(sh.first) << 20, np = bytes / piece;
          const int ns = sh.second;
          double pb[3] = {0, 0, 0};
          for (int rep = 0; rep < 4; ++rep) {
            for (int dir = 0; dir < 3; ++dir) {  // 0 H2D, 1 D2H, 2 both
              const double t0 = now_s();
              for (size_t i = 0; i < np; ++i) {
                if (dir != 1)
                  CK(hipMemcpyAsync(static_cast<char*>(d1) + i * piece, static_cast<char*>(h1) + i * piece, piece,
                                    hipMemcpyHostToDevice, ps[i % ns]));
                if (dir != 0)
                  CK(hipMemcpyAsync(static_cast<char*>(h2) + i * piece, static_cast<char*>(d2) + i * piece, piece,
                                    hipMemcpyDeviceToHost, ps[4 + i % ns]));
              }
              for (auto& x : ps) CK(hipStreamSynchronize(x));
              const double moved = (dir == 2 ? 2.0 : 1.0) * static_cast<double>(np * piece);
              if (rep > 0) pb[dir] = std::max(pb[dir], moved / (now_s() - t0) / 1e9);
            }
          }
          printf("{\"test\":\"pcie_pieces\",\"alloc\":\"%s\",\"piece_bytes\":%zu,\"streams_per_direction\":%d,"
                 "\"h2d_GBps\":%.1f,\"d2h_GBps\":%.1f,\"duplex_GBps\":%.1f}\n", names[f], piece, ns, pb[0], pb[1], pb[2]);
        }
        printf("{\"test\":\"pcie_in2_out1\",\"alloc\":\"%s\",\"piece_bytes\":%d,\"GBps\":%.1f}\n", names[f],
               8 << 20, pcie_in2_out1(d1, h1, d2, h2, bytes, ps[0], ps[4]));
        for (auto& x : ps) CK(hipStreamDestroy(x));
      }
      CK(hipHostFree(h1));
      CK(hipHostFree(h2));
    }
    CK(hipFree(d1));
    CK(hipFree(d2));
  } else if (what == "link") {
    // the copy path of the manager's piecewise transfers alone: pieces (8 MiB,
    // or the third argument in MiB) on one stream per direction between HBM
    // and non-coherent pinned memory (the staging kind), host to device,
    // device to host, both at once with equal bytes, and the 2:1 in/out mix
    const size_t bytes = (argc > 2 ? strtoull(argv[2], nullptr, 10) : 256) << 20;
    const size_t piece = (argc > 3 ? strtoull(argv[3], nullptr, 10) : 8) << 20;
    if (piece == 0 || bytes < piece || bytes % piece) {
      fprintf(stderr, "link: <MiB> must be a positive multiple of the piece size\n");
      return 1;
    }
    const size_t np = bytes / piece;
    void *d1, *d2, *h1, *h2;
    CK(hipMalloc(&d1, bytes));
    CK(hipMalloc(&d2, bytes));
    CK(hipMemset(d2, 2, bytes));
    CK(hipHostMalloc(&h1, bytes, hipHostMallocNonCoherent));
    CK(hipHostMalloc(&h2, bytes, hipHostMallocNonCoherent));
    memset(h1, 1, bytes);
    memset(h2, 2, bytes);
    hipStream_t in, out;
    CK(hipStreamCreateWithFlags(&in, hipStreamNonBlocking));
    CK(hipStreamCreateWithFlags(&out, hipStreamNonBlocking));
    double rate[3] = {0, 0, 0};
    for (int rep = 0; rep < 4; ++rep) {
      for (int dir = 0; dir < 3; ++dir) {  // 0 H2D, 1 D2H, 2 both
        const double t0 = now_s();
        for (size_t i = 0; i < np; ++i) {
          if (dir != 1)
            CK(hipMemcpyAsync(static_cast<char*>(d1) + i * piece, static_cast<char*>(h1) + i * piece, piece,
                              hipMemcpyHostToDevice, in));
          if (dir != 0)
            CK(hipMemcpyAsync(static_cast<char*>(h2) + i * piece, static_cast<char*>(d2) + i * piece, piece,
                              hipMemcpyDeviceToHost, out));
        }
        CK(hipStreamSynchronize(in));
        CK(hipStreamSynchronize(out));
        const double moved = (dir == 2 ? 2.0 : 1.0) * static_cast<double>(np * piece);
        if (rep > 0) rate[dir] = std::max(rate[dir], moved / (now_s() - t0) / 1e9);
      }
    }
    const double mix = pcie_in2_out1(d1, h1, d2, h2, bytes, in, out, piece);
    printf("{\"test\":\"link\",\"alloc\":\"noncoherent\",\"piece_bytes\":%zu,\"h2d_GBps\":%.1f,\"d2h_GBps\":%.1f,"
           "\"duplex_GBps\":%.1f,\"in2_out1_GBps\":%.1f}\n", piece, rate[0], rate[1], rate[2], mix);
    CK(hipStreamDestroy(in));
    CK(hipStreamDestroy(out));
    CK(hipHostFree(h1));
    CK(hipHostFree(h2));
    CK(hipFree(d1));
    CK(hipFree(d2));
  } else if (what == "hostcopy") {
    // CPU memcpy between pageable memory and pinned staging, as the manager's
    // copy engine does it: 1 and 8 threads, default and non-coherent pinned
    const size_t bytes = (argc > 2 ? strtoull(argv[2], nullptr, 10) : 512) << 20;
    const unsigned flag_sets[2] = {hipHostMallocDefault, hipHostMallocNonCoherent};
    const char* names[2] = {"default", "noncoherent"};
    char* pageable = static_cast<char*>(aligned_alloc(4096, bytes));
    memset(pageable, 3, bytes);
    for (int f = 0; f < 2; ++f) {
      char* pin = nullptr;
      CK(hipHostMalloc(reinterpret_cast<void**>(&pin), bytes, flag_sets[f]));
      memset(pin, 4, bytes);
      for (int nt : {1, 8}) {
        auto par = [&](char* dst, const char* src) {
          std::vector<std::thread> th;
          const size_t part = bytes / nt;
          for (int t = 0; t < nt; ++t)
            th.emplace_back([=] { memcpy(dst + t * part, src + t * part, part); });
          for (auto& x : th) x.join();
        };
        double in_best = 0, out_best = 0;
        for (int rep = 0; rep < 4; ++rep) {
          double t0 = now_s();
          par(pin, pageable);
          const double in = bytes / (now_s() - t0) / 1e9;
          t0 = now_s();
          par(pageable, pin);
          const double out = bytes / (now_s() - t0) / 1e9;
          if (rep > 0) {
            in_best = std::max(in_best, in);
            out_best = std::max(out_best, out);
          }
        }
        printf("{\"test\":\"hostcopy\",\"pinned\":\"%s\",\"threads\":%d,\"to_pinned_GBps\":%.1f,\"from_pinned_GBps\":%.1f}\n",
               names[f], nt, in_best, out_best);
      }
      CK(hipHostFree(pin));
    }
    free(pageable);
  } else if (what == "latency") {
    // launch -> completion observed by the host, for an empty kernel, by
    // event query, by stream synchronize, by a flag in pinned host memory
    // that a trailing kernel stores (vector store, system-scope release) and
    // by a flag that the stream itself writes (hipStreamWriteValue64); and
    // the cost of a 1.3 KiB kernel argument
    const int iters = argc > 2 ? atoi(argv[2]) : 2000;
    hipStream_t s;
    CK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t ev, te0, te1;
    CK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    CK(hipEventCreate(&te0));
    CK(hipEventCreate(&te1));
    uint32_t* flag = nullptr;
    CK(hipHostMalloc(reinterpret_cast<void**>(&flag), 4096, hipHostMallocDefault));
    *flag = 0;
    uint64_t* flag64 = reinterpret_cast<uint64_t*>(flag + 16);   // its own 64-byte line
    *flag64 = 0;
    void* flag64_dev = nullptr;
    CK(hipHostGetDevicePointer(&flag64_dev, flag64, 0));
    Big big;
    memset(&big, 0, sizeof(big));
    hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, s, 0);
    CK(hipStreamSynchronize(s));
    auto run = [&](int mode) {
      double t0 = now_s();
      for (int i = 0; i < iters; ++i) {
        if (mode == 5 || mode == 6 || mode == 8 || mode == 9) {
          // completion (and timing) events carried by the dispatch itself
          if (mode == 8) CK(hipEventRecord(te0, s));
          hipEvent_t stop = mode == 9 ? ev : te1;
          hipExtLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, s, mode == 6 ? te0 : nullptr, stop, 0, i);
          while (hipEventQuery(stop) == hipErrorNotReady) {
          }
          continue;
        }
        if (mode == 10) {   // timing marker after the launch only
          hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, s, i);
          CK(hipEventRecord(te1, s));
          while (hipEventQuery(te1) == hipErrorNotReady) {
          }
          continue;
        }
        if (mode == 7) CK(hipEventRecord(te0, s));   // the manager's pattern: markers around the launch
        if (mode == 3) hipLaunchKernelGGL(big_arg_kernel, dim3(1), dim3(64), 0, s, big);
        else hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, s, i);
        if (mode == 7) {
          CK(hipEventRecord(te1, s));
          while (hipEventQuery(te1) == hipErrorNotReady) {
          }
          continue;
        }
        if (mode == 0 || mode == 3) {
          CK(hipEventRecord(ev, s));
          while (hipEventQuery(ev) == hipErrorNotReady) {
          }
        } else if (mode == 1) {
          CK(hipStreamSynchronize(s));
        } else if (mode == 4) {
          CK(hipStreamWriteValue64(s, flag64_dev, static_cast<uint64_t>(i + 1), 0));
          while (__atomic_load_n(flag64, __ATOMIC_ACQUIRE) != static_cast<uint64_t>(i + 1)) {
          }
        } else {
          hipLaunchKernelGGL(signal_kernel, dim3(1), dim3(64), 0, s, flag, static_cast<uint32_t>(i + 1));
          while (__atomic_load_n(flag, __ATOMIC_ACQUIRE) != static_cast<uint32_t>(i + 1)) {
          }
        }
      }
      return (now_s() - t0) / iters * 1e6;
    };
    const double q = run(0), sy = run(1), wv = run(2), big_q = run(3), sw = run(4);
    const double ext_stop = run(5), ext_both = run(6), markers = run(7);
    const double marker_then_ext = run(8), ext_untimed = run(9), marker_after = run(10);
    printf("{\"test\":\"latency\",\"iters\":%d,\"event_query_us\":%.2f,\"stream_sync_us\":%.2f,"
           "\"host_flag_us\":%.2f,\"stream_write_value_us\":%.2f,\"big_arg_event_query_us\":%.2f,\"big_arg_bytes\":%zu,"
           "\"timed_markers_us\":%.2f,\"ext_launch_stop_event_us\":%.2f,\"ext_launch_start_stop_events_us\":%.2f,"
           "\"timed_marker_then_ext_launch_us\":%.2f,\"ext_launch_untimed_stop_us\":%.2f,\"timed_marker_after_us\":%.2f}\n",
           iters, q, sy, wv, sw, big_q, sizeof(Big), markers, ext_stop, ext_both, marker_then_ext, ext_untimed, marker_after);
    CK(hipHostFree(flag));
  } else {
    fprintf(stderr, "unknown test %s\n", what.c_str());
    return 1;
  }
  return 0;
}
