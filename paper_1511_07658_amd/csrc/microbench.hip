// Device ceilings of the MI355X the GVM runs on:
//   copy   <MiB> <reps>   plain device-to-device copy kernel (HBM read+write rate;
//                         also the reference kernel for scaling FETCH_SIZE/WRITE_SIZE)
//   mfma   <iters>        FP32 MFMA issue rate (v_mfma_f32_32x32x2_f32 chains)
//   pcie   <MiB>          pinned host<->device copy rates, one direction and both
//   init                  time to create the device context in a fresh process
// Prints one JSON object per test.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

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

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: %s copy <MiB> <reps> | mfma <iters> | pcie <MiB> | init\n", argv[0]);
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
    const size_t bytes = (argc > 2 ? strtoull(argv[2], nullptr, 10) : 256) << 20;
    void *h1, *h2, *d1, *d2;
    CK(hipHostMalloc(&h1, bytes, hipHostMallocDefault));
    CK(hipHostMalloc(&h2, bytes, hipHostMallocDefault));
    CK(hipMalloc(&d1, bytes));
    CK(hipMalloc(&d2, bytes));
    memset(h1, 1, bytes);
    memset(h2, 2, bytes);
    hipStream_t s1, s2;
    CK(hipStreamCreateWithFlags(&s1, hipStreamNonBlocking));
    CK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    CK(hipMemcpyAsync(d1, h1, bytes, hipMemcpyHostToDevice, s1));
    CK(hipStreamSynchronize(s1));
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
    printf("{\"test\":\"pcie_pinned\",\"bytes\":%zu,\"h2d_GBps\":%.1f,\"d2h_GBps\":%.1f,\"duplex_GBps\":%.1f}\n", bytes,
           h2d, d2h, both);
    CK(hipFree(d1));
    CK(hipFree(d2));
    CK(hipHostFree(h1));
    CK(hipHostFree(h2));
  } else {
    fprintf(stderr, "unknown test %s\n", what.c_str());
    return 1;
  }
  return 0;
}
