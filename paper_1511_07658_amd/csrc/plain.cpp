// The plain per-process path without virtualization: the single-process
// execution cycle of Section 4.1 (initialise the device and a context,
// allocate, send, compute, retrieve), run in the caller's own process with
// the same kernel code object the manager uses.
#include <hip/hip_runtime.h>

#include <cstring>

#include "common.hpp"
#include "gvm.h"
#include "kernels.hpp"

namespace {

double secs(uint64_t a, uint64_t b) { return (b - a) * 1e-9; }

#define PCHK(expr)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      if (dev) (void)hipFree(dev);                                                           \
      return gvm::fail(GVM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));              \
    }                                                                                     \
  } while (0)

}  // namespace

extern "C" int gvm_plain_run(int kernel_id, const void* in, void* out, uint64_t n, float bs_rate,
                             float bs_volatility, double* t) {
  gvm::clear_error();
  gvm::Layout lay;
  if (!gvm::request_layout(kernel_id, n, &lay)) return gvm::fail(GVM_EINVAL, "bad kernel id or size");
  if (!in || !out) return gvm::fail(GVM_EINVAL, "in/out is NULL");
  uint8_t* dev = nullptr;
  const uint64_t t0 = gvm::now_ns();
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return gvm::fail(GVM_EDEVICE, "no HIP device visible");
  PCHK(hipSetDevice(0));
  PCHK(hipFree(nullptr));  // creates the context
  hipDeviceProp_t prop;
  PCHK(hipGetDeviceProperties(&prop, 0));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return gvm::fail(GVM_EDEVICE, "device is not gfx950");
  const uint64_t t1 = gvm::now_ns();
  PCHK(hipMalloc(reinterpret_cast<void**>(&dev), gvm::slot_bytes(lay)));
  const uint64_t t2 = gvm::now_ns();
  PCHK(hipMemcpy(dev, in, lay.in_bytes, hipMemcpyHostToDevice));
  const uint64_t t3 = gvm::now_ns();
  float* fin = reinterpret_cast<float*>(dev);
  float* fout = reinterpret_cast<float*>(dev + gvm::slot_out_offset(lay));
  hipError_t e = hipSuccess;
  if (kernel_id == GVM_K_VECADD || kernel_id == GVM_K_VECMUL) {
    gvm::VecGroup g{};
    g.count = 1;
    g.d[0] = gvm::VecDesc{fin, fin + n, fout, n, 0};
    gvm::finalize_vec_group(g);
    e = kernel_id == GVM_K_VECADD ? gvm::launch_vecadd_group(g, nullptr) : gvm::launch_vecmul_group(g, nullptr);
  } else if (kernel_id == GVM_K_BLACKSCHOLES) {
    gvm::BsGroup g{};
    g.count = 1;
    g.rate = bs_rate;
    g.volatility = bs_volatility;
    g.d[0] = gvm::BsDesc{fin, fin + n, fin + 2 * n, fout, fout + n, n, 0};
    gvm::finalize_bs_group(g);
    e = gvm::launch_bs_group(g, nullptr);
  } else if (kernel_id == GVM_K_EP) {
    gvm::EpGroup g{};
    g.count = 1;
    g.d[0] = gvm::EpDesc{reinterpret_cast<const uint64_t*>(dev), reinterpret_cast<uint64_t*>(fout),
                         reinterpret_cast<uint64_t*>(dev + gvm::slot_scratch_offset(lay)), n, 0, 0};
    gvm::finalize_ep_group(g);
    e = gvm::launch_ep_group(g, nullptr);
  } else {
    gvm::GemmGroup g{};
    g.count = 1;
    g.d[0] = gvm::GemmDesc{fin, fin + n * n, fout, static_cast<uint32_t>(n), 0, 0, 0};
    const int c = gvm::gemm_config_for(n);
    gvm::finalize_gemm_group(g, c);
    e = gvm::launch_sgemm_group(g, c, nullptr);
  }
  PCHK(e);
  PCHK(hipDeviceSynchronize());
  const uint64_t t4 = gvm::now_ns();
  PCHK(hipMemcpy(out, dev + gvm::slot_out_offset(lay), lay.out_bytes, hipMemcpyDeviceToHost));
  const uint64_t t5 = gvm::now_ns();
  PCHK(hipFree(dev));
  dev = nullptr;
  const uint64_t t6 = gvm::now_ns();
  if (t) {
    t[0] = secs(t0, t1);
    t[1] = secs(t1, t2);
    t[2] = secs(t2, t3);
    t[3] = secs(t3, t4);
    t[4] = secs(t4, t5);
    t[5] = secs(t5, t6);
  }
  return GVM_OK;
}
