// Shared-memory protocol between rank processes and the manager.
//
// Section 5 builds the base layer from one POSIX shared-memory space per
// process (the data) plus POSIX message queues (requests in, handshake
// responses out).  Here the queues are single-producer single-consumer rings
// that live in shared memory next to a futex doorbell, so that a request or a
// response costs no system call while the other side is awake.
//
// Objects of namespace NAME:
//   /NAME.ctl   control segment: CtlHeader, then one RankSlot per rank
//   /NAME.rK    rank K's data space (shm_bytes_per_rank bytes)
#pragma once

#include <atomic>
#include <cstdint>
#include <string>

#include "gvm.h"

namespace gvm {

constexpr uint64_t kMagic = 0x31564d47534d5647ull;  // "GVMSGMV1"
constexpr uint32_t kVersion = 2;
constexpr uint32_t kRingCap = 64;  // entries, power of two
constexpr int kMaxRanks = 256;

// Message kinds carried in Request::kernel_id besides the gvm_kernel ids.
constexpr uint32_t kMsgAttach = 0x100;
constexpr uint32_t kMsgDetach = 0x101;

enum CtlState : uint32_t { kStarting = 0, kReady = 1, kStopping = 2, kStopped = 3 };
enum SlotState : uint32_t { kSlotFree = 0, kSlotClaimed = 1, kSlotAttached = 2 };

struct Request {        // 64 bytes
  uint64_t ticket;
  uint32_t kernel_id;
  uint32_t flags;
  uint64_t n;
  uint64_t off_in;      // byte offset of the input in the rank's data space
  uint64_t off_out;     // byte offset of the output in the rank's data space
  uint64_t in_bytes;
  uint64_t out_bytes;
  uint64_t t_submit_ns;
};
static_assert(sizeof(Request) == 64, "Request must be 64 bytes");

struct Response {       // 64 bytes
  uint64_t ticket;
  int32_t status;
  uint32_t kernel_id;
  uint64_t t_submit_ns;
  uint64_t t_admit_ns;   // manager admitted the request
  uint64_t t_launch_ns;  // manager enqueued its device work
  uint64_t t_device_ns;  // device work observed complete
  uint64_t t_done_ns;    // result in the data space, response posted
  uint64_t reserved;
};
static_assert(sizeof(Response) == 64, "Response must be 64 bytes");

template <class T>
struct Ring {
  alignas(64) std::atomic<uint64_t> head;  // next entry to consume (consumer writes)
  alignas(64) std::atomic<uint64_t> tail;  // next entry to produce (producer writes)
  alignas(64) T slots[kRingCap];

  void reset() {
    head.store(0, std::memory_order_relaxed);
    tail.store(0, std::memory_order_relaxed);
  }
  bool push(const T& v) {
    const uint64_t t = tail.load(std::memory_order_relaxed);
    if (t - head.load(std::memory_order_acquire) >= kRingCap) return false;
    slots[t & (kRingCap - 1)] = v;
    tail.store(t + 1, std::memory_order_release);
    return true;
  }
  bool pop(T* v) {
    const uint64_t h = head.load(std::memory_order_relaxed);
    if (h == tail.load(std::memory_order_acquire)) return false;
    *v = slots[h & (kRingCap - 1)];
    head.store(h + 1, std::memory_order_release);
    return true;
  }
  bool empty() const { return head.load(std::memory_order_acquire) == tail.load(std::memory_order_acquire); }
  bool full() const {
    return tail.load(std::memory_order_acquire) - head.load(std::memory_order_acquire) >= kRingCap;
  }
};

// What a rank waiting for a response is doing (RankSlot::rank_sleeping).
enum RankSleep : uint32_t { kAwake = 0, kSleepOwnBell = 1, kSleepGroupBell = 2 };

struct RankSlot {
  alignas(64) std::atomic<uint32_t> state;   // SlotState
  std::atomic<int32_t> pid;                  // owning process
  std::atomic<uint32_t> epoch;               // bumped by every attach
  alignas(64) std::atomic<uint32_t> resp_bell;      // futex: manager -> rank
  std::atomic<uint32_t> rank_sleeping;       // kAwake, kSleepOwnBell or kSleepGroupBell
  Ring<Request> req;                         // rank -> manager
  Ring<Response> resp;                       // manager -> rank
};

struct CtlHeader {
  uint64_t magic;
  uint32_t version;
  uint32_t nranks;
  uint64_t shm_bytes_per_rank;
  uint64_t slot_stride;                      // bytes between RankSlots
  alignas(64) std::atomic<uint32_t> state;   // CtlState
  std::atomic<int32_t> manager_pid;
  std::atomic<uint32_t> generation;
  std::atomic<uint64_t> heartbeat_ns;
  alignas(64) std::atomic<uint32_t> bell;    // futex: ranks -> manager
  std::atomic<uint32_t> manager_sleeping;
  // futex: manager -> every rank that sleeps on it.  In batch mode the ranks
  // of a batch are answered together, so they sleep on this one word and a
  // single wake-up call reaches all of them.
  alignas(64) std::atomic<uint32_t> group_bell;
  alignas(64) gvm_config cfg;
};

inline uint64_t ctl_slot_stride() { return (sizeof(RankSlot) + 63) / 64 * 64; }
inline uint64_t ctl_bytes(uint32_t nranks) {
  return (sizeof(CtlHeader) + 63) / 64 * 64 + static_cast<uint64_t>(nranks) * ctl_slot_stride();
}
inline RankSlot* ctl_slot(CtlHeader* h, int rank) {
  auto* base = reinterpret_cast<uint8_t*>(h) + (sizeof(CtlHeader) + 63) / 64 * 64;
  return reinterpret_cast<RankSlot*>(base + static_cast<uint64_t>(rank) * h->slot_stride);
}

std::string ctl_object_name(const std::string& ns);
std::string data_object_name(const std::string& ns, int rank);
std::string default_namespace();

// A mapped POSIX shared-memory object.
struct Segment {
  void* addr = nullptr;
  uint64_t bytes = 0;
  std::string name;
  bool owner = false;

  int create(const std::string& name, uint64_t bytes);   // creates (replacing a stale one) and maps
  int open(const std::string& name);                      // maps an existing object (its full size)
  void close();                                           // unmaps; unlinks if owner
  ~Segment() { close(); }
};

}  // namespace gvm
