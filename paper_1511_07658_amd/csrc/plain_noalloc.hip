// Allocation-free variant of the plain per-process path: the same kernel code
// objects as gvm_plain_run on caller-owned device buffers, enqueued on the
// caller's stream, for callers that cannot allocate device memory.  The only
// device memory beyond the caller's input and output is the EP-like kernel's
// per-unit partial records, which live in one static device array per GPU.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "common.hpp"
#include "gvm.h"
#include "kernels.hpp"

namespace {

constexpr uint64_t kScratchWords = GVM_NOALLOC_SCRATCH_BYTES / sizeof(uint64_t);
static_assert(GVM_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch is a whole number of 256-byte blocks");

// Partial records of the EP-like kernel (one per work unit of kEpUnit pairs).
// Every call on a GPU shares that GPU's copy and leaves its contents behind;
// the unit launch writes every record the reduce launch reads, so nothing has
// to start at zero.  In host code `scratch` names a host-side stand-in: its
// device address is taken once per device with hipGetSymbolAddress.
__device__ __align__(256) uint64_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint64_t* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device
bool g_checked[kMaxDevices] = {};       // device is a gfx950

// The device address of `scratch` on the current device (looked up on the
// first call with that device current), or null with the error recorded.
uint64_t* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_checked[dev]) {
    hipDeviceProp_t prop;
    const hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
      gvm::fail(GVM_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
      return nullptr;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      gvm::fail(GVM_EDEVICE, "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
      return nullptr;
    }
    g_checked[dev] = true;
  }
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      gvm::fail(GVM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return nullptr;
    }
    g_scratch[dev] = static_cast<uint64_t*>(p);
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" int gvm_plain_run_noalloc(int kernel_id, const void* d_in, void* d_out, uint64_t n, float bs_rate,
                                     float bs_volatility, void* stream) {
  gvm::clear_error();
  gvm::Layout lay;
  if (!gvm::request_layout(kernel_id, n, &lay)) return gvm::fail(GVM_EINVAL, "bad kernel id or size");
  if (!d_in || !d_out) return gvm::fail(GVM_EINVAL, "d_in/d_out is NULL");
  if (kernel_id == GVM_K_EP && lay.scratch_bytes > GVM_NOALLOC_SCRATCH_BYTES)
    return gvm::fail(GVM_ENOMEM, "EP request of %llu pairs needs %llu bytes of scratch; the static scratch holds %u",
                     (unsigned long long)n, (unsigned long long)lay.scratch_bytes, GVM_NOALLOC_SCRATCH_BYTES);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return gvm::fail(GVM_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return gvm::fail(GVM_EDEVICE, "device index %d beyond %d", dev, kMaxDevices);
  uint64_t* part = scratch_on(dev);
  if (!part) return GVM_EDEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float* fin = static_cast<const float*>(d_in);
  float* fout = static_cast<float*>(d_out);
  if (kernel_id == GVM_K_VECADD || kernel_id == GVM_K_VECMUL) {
    gvm::VecGroup g{};
    g.count = 1;
    g.d[0] = gvm::VecDesc{fin, fin + n, fout, n, 0};
    gvm::finalize_vec_group(g);
    e = kernel_id == GVM_K_VECADD ? gvm::launch_vecadd_group(g, s) : gvm::launch_vecmul_group(g, s);
  } else if (kernel_id == GVM_K_BLACKSCHOLES) {
    gvm::BsGroup g{};
    g.count = 1;
    g.rate = bs_rate;
    g.volatility = bs_volatility;
    g.d[0] = gvm::BsDesc{fin, fin + n, fin + 2 * n, fout, fout + n, n, 0};
    gvm::finalize_bs_group(g);
    e = gvm::launch_bs_group(g, s);
  } else if (kernel_id == GVM_K_EP) {
    gvm::EpGroup g{};
    g.count = 1;
    g.d[0] = gvm::EpDesc{static_cast<const uint64_t*>(d_in), static_cast<uint64_t*>(d_out), part, n, 0, 0};
    gvm::finalize_ep_group(g);
    e = gvm::launch_ep_group(g, s);
  } else {
    gvm::GemmGroup g{};
    g.count = 1;
    g.d[0] = gvm::GemmDesc{fin, fin + n * n, fout, static_cast<uint32_t>(n), 0, 0, 0};
    const int c = gvm::gemm_config_for(n);
    gvm::finalize_gemm_group(g, c);
    e = gvm::launch_sgemm_group(g, c, s);
  }
  if (e != hipSuccess) return gvm::fail(GVM_EDEVICE, "kernel launch: %s", hipGetErrorString(e));
  return GVM_OK;
}
