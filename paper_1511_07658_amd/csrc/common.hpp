// Shared helpers of the GVM library: status/error text, clocks, request
// layouts, futex doorbells.
#pragma once

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <string>

#include "gvm.h"

namespace gvm {

// Thread-local last error.  Returns `code` so callers can `return fail(...)`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
const char* last_error_text();
void clear_error();

uint64_t now_ns();  // CLOCK_MONOTONIC, shared by every process on the host

constexpr uint64_t kAlign = 256;  // device / staging sub-buffer alignment
inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Packed binary32 layout of one request (bytes of `in` and `out`).
struct Layout {
  uint64_t in_bytes = 0;
  uint64_t out_bytes = 0;
  uint64_t scratch_bytes = 0;  // device-only working space after the output (never copied)
};

constexpr int kNumKernelIds = 6;  // kernel ids 1..5; index 0 collects mixed graph launches

// Requests move between the ranks' shared memory, the pinned staging and the
// device in pieces of this size (unless batch_timing asks for whole copies):
// each piece's next hop starts as soon as it lands.
// Bytes of one piece of a piecewise copy: set by the manager at init (32 MiB
// in batch mode, 8 MiB in serving mode); GVM_PIECE_MB, read once, overrides
// with 1..64.
uint64_t piece_bytes();
void set_piece_bytes(uint64_t bytes);
inline uint32_t piece_count(uint64_t bytes) { return static_cast<uint32_t>((bytes + piece_bytes() - 1) / piece_bytes()); }

// A request whose copies total at most this many bytes keeps them on the
// stream that runs its kernel: such a copy takes ~18 us on the link, less
// than a dependency between two hardware queues costs (~15-20 us), and it
// gains nothing from the copy FIFOs.
// CU partition for serving QoS (gvm_config.latency_cus), on a device of
// kPartitionCus CUs: bit i of a mask is CU i in HIP's numbering.  Write
// i = 32a + 8b + c with c = i % 8, b = (i / 8) % 4 and a = i / 32.  The
// latency partition of 32m CUs (m = 1..7) takes:
//  * every CU with b < m / 2;
//  * for odd m, also those with b == m / 2 and a + c even.
// The bulk partition takes the rest.  Whether the 8 XCDs own CUs by i % 8
// (interleaved) or by i / 32 (contiguous), every XCD then holds the same
// share of each partition.  No queue is left with an XCD whose workgroups
// could never be placed.  Fills kPartitionCus / 32 words of each mask;
// GVM_EINVAL for other values of latency_cus.
constexpr int kPartitionCus = 256;
int cu_partition_masks(uint32_t latency_cus, uint32_t* latency_mask, uint32_t* bulk_mask);

constexpr uint64_t kLocalCopyBytes = 1ull << 20;

// EP-like kernel: pairs per work unit, and the 64-bit words of one result
// record (sx, sy, q[0..9]), the request's output and each unit's partial.
constexpr uint64_t kEpUnit = 1ull << 15;
constexpr uint64_t kEpWords = 12;
// false if the kernel id is unknown, n == 0 or the size overflows.
bool request_layout(int kernel_id, uint64_t n, Layout* out);
// Device slot of a request: input, then output at the next aligned offset,
// then the device-only scratch at the next aligned offset.
inline uint64_t slot_bytes(const Layout& l) {
  return align_up(l.in_bytes, kAlign) + align_up(l.out_bytes, kAlign) + align_up(l.scratch_bytes, kAlign);
}
inline uint64_t slot_out_offset(const Layout& l) { return align_up(l.in_bytes, kAlign); }
inline uint64_t slot_scratch_offset(const Layout& l) { return align_up(l.in_bytes, kAlign) + align_up(l.out_bytes, kAlign); }

// Futex on a 32-bit word that lives in shared memory (process-shared).
// Returns 0 when woken or the value differed, GVM_ETIMEDOUT on timeout.
int futex_wait(std::atomic<uint32_t>* word, uint32_t expected, int64_t timeout_ns);
void futex_wake_all(std::atomic<uint32_t>* word);

bool pid_alive(int32_t pid);

// Spin budget (ns) read from an environment variable given in microseconds.
uint64_t spin_env_ns(const char* var, uint64_t default_us);

inline const char* kernel_name(int k) {
  switch (k) {
    case GVM_K_VECADD: return "vecadd";
    case GVM_K_BLACKSCHOLES: return "blackscholes";
    case GVM_K_SGEMM: return "sgemm";
    case GVM_K_VECMUL: return "vecmul";
    case GVM_K_EP: return "ep";
    default: return "unknown";
  }
}

}  // namespace gvm
