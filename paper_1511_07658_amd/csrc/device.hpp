// Device side of the manager: the GPU resources of Section 5 (one context,
// streams, per-process device and pinned host memory, prepared kernels) and
// the enqueue policies of Section 4.2.1.
#pragma once

#include <atomic>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "shm.hpp"

namespace gvm {

// Stages of an admitted request in the manager.
enum JobStage : int { kStageCopyIn = 0, kStageReady = 1, kStageDevice = 2, kStageCopyOut = 3 };

// One admitted request on its way through the device.  The manager moves its
// input shm -> pinned before launch() and its result pinned -> shm after the
// device work; the Device only moves pinned <-> device memory.
struct Job {
  int rank = -1;
  Request req{};
  Layout lay{};
  uint8_t* shm = nullptr;       // rank's data space (host)
  uint8_t* slot = nullptr;      // rank's device buffer: input at 0, output at slot_out_offset
  uint8_t* pin = nullptr;       // rank's pinned staging: same layout as the slot
  bool copy_in = true;
  bool copy_out = true;
  int status = GVM_OK;
  uint64_t t_admit_ns = 0;
  uint64_t t_launch_ns = 0;
  uint64_t t_device_ns = 0;
  void* batch = nullptr;        // device-private bookkeeping
  int done_index = -1;
  int stage = kStageCopyIn;
  std::atomic<int> copies{0};   // host copy chunks still in flight
  // Piecewise copies (piece_bytes()): the input's pieces go to the device as
  // each lands in the pinned staging, the output's pieces come back to shared
  // memory as each leaves the device.
  bool local = false;            // small copies: on the kernel's own stream, whole
  bool pieces = false;
  uint32_t in_pieces = 0, in_sent = 0;                 // input pieces; those whose H2D is queued
  std::unique_ptr<std::atomic<int>[]> in_pending;      // host copy chunks in flight per input piece
  uint32_t out_pieces = 0, out_taken = 0;              // output pieces; those handed to the host copy
  void* in_done = nullptr;       // device-private: marks the last input piece on the copy FIFO
  int part = -1;                 // CU partition of its kernel (latency_cus): 0 latency class, 1 the rest
  bool small = false;            // serving: a small request (small_request_bytes), staging copies first
  // serving: a rank's second request in flight has a device slot of its own
  // (freed when it is answered) and the staging region after the first's
  bool extra_slot = false;
  uint64_t extra_off = 0, extra_size = 0;
  uint64_t pin_off = 0, pin_len = 0;  // region of the rank's pinned staging it uses
};

struct KernelStats {
  uint64_t launches = 0;
  uint64_t requests = 0;
  double device_ms = 0.0;       // sum of launch durations from device events
  double work_flop = 0.0;       // algorithmic FLOP of the launched requests
  double work_bytes = 0.0;      // algorithmic HBM bytes of the launched requests
};

// Algorithmic work of one request (the per-unit figures: 12 B per vector
// element, 20 B per option, 2 n^3 FLOP and 12 n^2 compulsory bytes per GEMM,
// the 112 input and output bytes of an EP request, whose work is its n pairs).
void request_work(int kernel_id, uint64_t n, double* flop, double* bytes);

// Rough device time of one request on the whole MI355X (us), from its
// algorithmic work at sustained rates (FP32 MFMA 110 TFLOP/s, HBM 5 TB/s,
// 120 G EP pairs/s); it only sorts requests into the latency class.
double estimate_device_us(int kernel_id, uint64_t n);
constexpr double kLatencyClassUs = 50.0;

class Device {
 public:
  virtual ~Device() = default;
  virtual int open(const gvm_config& cfg) = 0;
  virtual uint8_t* arena() = 0;                 // hbm_budget_bytes of device memory
  virtual uint8_t* staging(int rank) = 0;       // pinned staging of a rank (nullptr on failure)
  // Queue the host-to-device copy of input bytes [off, off + bytes) of a
  // piecewise job (in order, before launch()).
  virtual int stream_in(Job* j, uint64_t off, uint64_t bytes) = 0;
  // Enqueue the device work of the admitted jobs under `policy` (a piecewise
  // job's copy-in is already queued; its copy-out is queued piece by piece).
  virtual int launch(std::vector<Job*>& jobs, int policy) = 0;
  // Leading output pieces of a piecewise job that have reached the pinned
  // staging (< 0 on a device error).
  virtual int out_pieces_done(Job* j) = 0;
  // 1 when the job's device work has finished, 0 if not yet, < 0 on a device error.
  virtual int query(Job* j) = 0;
  // Start a polling round: query() may then ask the runtime about each
  // completion event at most once until the next round.
  virtual void begin_poll() {}
  // After query() == 1: release the device bookkeeping of the job (the
  // result is in the pinned staging).  A batch whose last job finished is
  // retired later, by flush_retired().
  virtual void finish(Job* j) = 0;
  // Retire finished batches: read their device timings into the counters
  // and recycle their events.  Returns true if any batch was retired.  The
  // manager calls it while the device is busy or it is idle, so that this
  // work never delays answering the ranks.
  virtual bool flush_retired() { return false; }
  virtual void drain() = 0;
  virtual void close() = 0;
  virtual const KernelStats* kernel_stats() const = 0;  // indexed by kernel id (kNumKernelIds entries)
  virtual void reset_stats() = 0;
  virtual std::string describe() const = 0;
  // Batch device phases and copy timings (batch_timing), as a JSON object.
  virtual std::string timing_json() const { return "{}"; }
};

std::unique_ptr<Device> make_hip_device();
std::unique_ptr<Device> make_loopback_device();

}  // namespace gvm
