// Rank side of the C-ABI: the API layer of Section 5 (REQ / SND / STR / STP /
// RCV / RLS) over shared-memory rings.  Rank processes never touch the GPU.
#include <immintrin.h>
#include <sched.h>
#include <unistd.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "rank.hpp"
#include "shm.hpp"

namespace gvm {

namespace {

// Copy between the caller's memory and its shared-memory space.  A large
// copy is split over a few threads when the host has cores to spare: one
// thread moves about 10 GB/s, the PCIe link behind the manager ~57 GB/s.
// Threads per copy: the cores per rank (online CPUs / (ranks + 2)), 1..8.
void rank_copy(void* dst, const void* src, uint64_t bytes, uint32_t nranks) {
  constexpr uint64_t kSplit = 8ull << 20;
  static const long ncpu = sysconf(_SC_NPROCESSORS_ONLN);
  const long spare = ncpu / (static_cast<long>(nranks) + 2);
  const int nt = static_cast<int>(std::min<long>(std::min<long>(spare, 8), static_cast<long>(bytes / kSplit)));
  if (nt <= 1) {
    memcpy(dst, src, bytes);
    return;
  }
  const uint64_t part = (bytes / nt + 4095) & ~4095ull;
  std::vector<std::thread> ts;
  for (int i = 1; i < nt; ++i) {
    const uint64_t off = part * i;
    if (off >= bytes) break;
    ts.emplace_back([=] { memcpy(static_cast<uint8_t*>(dst) + off, static_cast<const uint8_t*>(src) + off, std::min(part, bytes - off)); });
  }
  memcpy(dst, src, std::min(part, bytes));
  for (auto& t : ts) t.join();
}

struct Alloc {
  uint64_t start, end;
  uint64_t ticket;
  bool freed;
};

struct Pending {
  uint64_t ticket;
  void* out;
  uint64_t off_out;
  uint64_t out_bytes;
  bool copy_out;
  uint32_t kernel_id;
};

struct RankHandle {
  std::mutex mu;
  bool attached = false;
  int rank = -1;
  RankSlot* slot = nullptr;
  Segment data;
  uint64_t next_ticket = 1;
  uint64_t user_region = 0;
  uint64_t head = 0;                 // next free byte of the ring allocator
  std::deque<Alloc> allocs;          // live reservations, oldest first
  std::deque<Pending> pending;       // submitted, result not yet received
  std::unordered_map<uint64_t, int> finished;  // received, not yet waited for
  std::unordered_map<uint64_t, Response> timing;  // responses of finished requests
};

// The control segment of the namespace this process's ranks use.
struct Namespace {
  std::mutex mu;
  std::string name;
  Segment ctl;
  CtlHeader* hdr = nullptr;
  int refs = 0;
};

Namespace g_ns;
RankHandle g_ranks[kMaxRanks];

bool manager_gone(CtlHeader* h) {
  const uint32_t st = h->state.load(std::memory_order_acquire);
  if (st == kStopping || st == kStopped) return true;
  const int32_t pid = h->manager_pid.load(std::memory_order_relaxed);
  return pid != getpid() && !pid_alive(pid);
}

void ring_manager(CtlHeader* h) {
  std::atomic_thread_fence(std::memory_order_seq_cst);
  h->bell.fetch_add(1, std::memory_order_seq_cst);
  if (h->manager_sleeping.load(std::memory_order_seq_cst)) futex_wake_all(&h->bell);
}

// ---- ring allocator over [user_region, size) of the data space ----

bool reserve(RankHandle& h, uint64_t bytes, uint64_t ticket, uint64_t* off) {
  const uint64_t size = h.data.bytes;
  const uint64_t lo = h.user_region;
  if (bytes == 0) {
    *off = 0;
    return true;
  }
  if (h.allocs.empty()) h.head = lo;
  uint64_t start;
  if (h.allocs.empty()) {
    if (lo + bytes > size) return false;
    start = lo;
  } else {
    const uint64_t tail = h.allocs.front().start;
    if (h.head >= tail) {  // not wrapped: free space is [head, size) and [lo, tail)
      if (h.head + bytes <= size) start = h.head;
      else if (lo + bytes <= tail) start = lo;
      else return false;
    } else {               // wrapped: free space is [head, tail)
      if (h.head + bytes <= tail) start = h.head;
      else return false;
    }
  }
  h.allocs.push_back(Alloc{start, start + bytes, ticket, false});
  h.head = start + bytes;
  *off = start;
  return true;
}

void release(RankHandle& h, uint64_t ticket) {
  for (auto& a : h.allocs)
    if (a.ticket == ticket) a.freed = true;
  while (!h.allocs.empty() && h.allocs.front().freed) h.allocs.pop_front();
  if (h.allocs.empty()) h.head = h.user_region;
}

// Move every posted response into `finished`, delivering results.
void drain(RankHandle& h) {
  Response r;
  while (h.slot->resp.pop(&r)) {
    for (auto it = h.pending.begin(); it != h.pending.end(); ++it) {
      if (it->ticket != r.ticket) continue;
      if (r.status == GVM_OK && it->copy_out)
        rank_copy(it->out, static_cast<uint8_t*>(h.data.addr) + it->off_out, it->out_bytes, g_ns.hdr ? g_ns.hdr->nranks : 1);
      release(h, it->ticket);
      h.pending.erase(it);
      break;
    }
    h.finished[r.ticket] = r.status;
    if (h.timing.size() < 4096) h.timing[r.ticket] = r;
  }
}

// Block until `done()` holds, a response arrives for it, or the deadline.
// Poll budget before a futex sleep: 1 ms when every rank and the manager can
// have a core of their own (longer than a typical synchronous step, so that
// the first rank to submit does not fall asleep and then wake last, a
// futex wake-up later), 10 us when the host is oversubscribed (a spinning
// rank would then steal the core of the one it waits for).
uint64_t rank_spin_ns(const CtlHeader* hdr) {
  if (getenv("GVM_RANK_SPIN_US")) return spin_env_ns("GVM_RANK_SPIN_US", 1000);
  static const long ncpu = sysconf(_SC_NPROCESSORS_ONLN);
  return (static_cast<long>(hdr->nranks) + 2 > ncpu) ? 10000ull : 1000000ull;
}

template <class Pred>
int wait_until(RankHandle& h, CtlHeader* hdr, int64_t timeout_ns, Pred done) {
  const uint64_t t0 = now_ns();
  const uint64_t spin = rank_spin_ns(hdr);
  const uint64_t deadline = timeout_ns < 0 ? UINT64_MAX : t0 + static_cast<uint64_t>(timeout_ns);
  uint32_t polls = 0;
  for (;;) {
    drain(h);
    if (done()) return GVM_OK;
    // the liveness probe is a system call: every 64th poll while polling
    if ((polls & 63) == 0 && manager_gone(hdr)) {
      drain(h);
      if (done()) return GVM_OK;
      return fail(GVM_EDEAD, "the GVM manager is gone");
    }
    const uint64_t now = now_ns();
    if (now >= deadline) return fail(GVM_ETIMEDOUT, "timed out");
    if (now - t0 < spin) {  // poll before sleeping (GVM_RANK_SPIN_US)
      for (int i = 0; i < 8; ++i) _mm_pause();
      // Give the core away now and then: a rank woken from its futex can be
      // placed on the manager's core, and a poll that never yields would
      // then hold off the manager (and the rank's own next request) for the
      // whole poll budget.
      if (++polls % 32 == 0) sched_yield();
      continue;
    }
    polls = 0;  // after a sleep: probe liveness on the next poll
    // batch mode: sleep on the shared group doorbell (one wake-up call per
    // answered batch); serving mode: on the rank's own doorbell
    const bool group = hdr->cfg.mode == GVM_MODE_BATCH;
    std::atomic<uint32_t>* bell = group ? &hdr->group_bell : &h.slot->resp_bell;
    const uint32_t v = bell->load(std::memory_order_acquire);
    h.slot->rank_sleeping.store(group ? kSleepGroupBell : kSleepOwnBell, std::memory_order_seq_cst);
    std::atomic_thread_fence(std::memory_order_seq_cst);
    if (h.slot->resp.empty()) {
      uint64_t left = deadline - now;
      futex_wait(bell, v, static_cast<int64_t>(std::min<uint64_t>(left, 50000000ull)));
    }
    h.slot->rank_sleeping.store(kAwake, std::memory_order_relaxed);
  }
}

int push_message(RankHandle& h, CtlHeader* hdr, const Request& m) {
  for (;;) {
    if (h.slot->req.push(m)) {
      ring_manager(hdr);
      return GVM_OK;
    }
    if (manager_gone(hdr)) return fail(GVM_EDEAD, "the GVM manager is gone");
    sched_yield();
  }
}

int map_namespace(const char* name) {
  std::string ns = (name && name[0]) ? std::string(name) : std::string();
  if (ns.empty()) {
    const char* env = getenv("GVM_NAME");
    ns = (env && env[0]) ? std::string(env) : default_namespace();
  }
  std::lock_guard<std::mutex> lk(g_ns.mu);
  if (g_ns.refs > 0) {
    if (g_ns.name != ns) return fail(GVM_ESTATE, "ranks of this process are attached to namespace %s", g_ns.name.c_str());
    ++g_ns.refs;
    return GVM_OK;
  }
  // wait up to 10 s for the manager to publish the namespace
  const uint64_t t0 = now_ns();
  int rc = GVM_ESYS;
  while (now_ns() - t0 < 10000000000ull) {
    rc = g_ns.ctl.open(ctl_object_name(ns));
    if (rc == GVM_OK) {
      auto* h = static_cast<CtlHeader*>(g_ns.ctl.addr);
      if (g_ns.ctl.bytes >= sizeof(CtlHeader) && h->magic == kMagic && h->version == kVersion &&
          h->state.load(std::memory_order_acquire) == kReady && g_ns.ctl.bytes >= ctl_bytes(h->nranks))
        break;
      g_ns.ctl.close();
      rc = GVM_ESTATE;
    }
    usleep(2000);
  }
  if (rc != GVM_OK) return fail(rc == GVM_ESTATE ? GVM_ESTATE : GVM_ESYS, "no ready GVM manager in namespace %s", ns.c_str());
  g_ns.hdr = static_cast<CtlHeader*>(g_ns.ctl.addr);
  g_ns.name = ns;
  g_ns.refs = 1;
  return GVM_OK;
}

void unmap_namespace() {
  std::lock_guard<std::mutex> lk(g_ns.mu);
  if (g_ns.refs > 0 && --g_ns.refs == 0) {
    g_ns.ctl.close();
    g_ns.hdr = nullptr;
    g_ns.name.clear();
  }
}

}  // namespace

int rank_attach(const char* name, int rank) {
  if (rank < 0 || rank >= kMaxRanks) return fail(GVM_EINVAL, "rank %d out of range", rank);
  RankHandle& h = g_ranks[rank];
  std::lock_guard<std::mutex> lk(h.mu);
  if (h.attached) return fail(GVM_ESTATE, "rank %d is already attached by this process", rank);
  int rc = map_namespace(name);
  if (rc != GVM_OK) return rc;
  CtlHeader* hdr = g_ns.hdr;
  if (static_cast<uint32_t>(rank) >= hdr->nranks) {
    unmap_namespace();
    return fail(GVM_EINVAL, "rank %d >= nranks %u", rank, hdr->nranks);
  }
  RankSlot* s = ctl_slot(hdr, rank);
  // claim the VGPU; a slot left by a dead process is freed by the manager
  const uint64_t t0 = now_ns();
  for (;;) {
    uint32_t expect = kSlotFree;
    if (s->state.compare_exchange_strong(expect, kSlotClaimed, std::memory_order_acq_rel)) break;
    const int32_t owner = s->pid.load(std::memory_order_acquire);
    if (owner != 0 && pid_alive(owner) ) {
      unmap_namespace();
      return fail(GVM_ESTATE, "rank %d is attached by live process %d", rank, owner);
    }
    if (now_ns() - t0 > 5000000000ull || manager_gone(hdr)) {
      unmap_namespace();
      return fail(GVM_ESTATE, "rank %d slot was not released", rank);
    }
    usleep(1000);
  }
  s->pid.store(getpid(), std::memory_order_release);
  s->epoch.fetch_add(1);
  s->resp.head.store(s->resp.tail.load(std::memory_order_acquire), std::memory_order_release);  // drop stale responses
  rc = h.data.open(data_object_name(g_ns.name, rank));
  if (rc != GVM_OK) {
    s->pid.store(0);
    s->state.store(kSlotFree, std::memory_order_release);
    unmap_namespace();
    return rc;
  }
  h.slot = s;
  h.rank = rank;
  h.pending.clear();
  h.finished.clear();
  h.timing.clear();
  h.allocs.clear();
  h.user_region = 0;
  h.head = 0;
  h.next_ticket = 1;
  Request m{};
  m.kernel_id = kMsgAttach;
  m.ticket = 0;
  m.t_submit_ns = now_ns();
  rc = push_message(h, hdr, m);
  if (rc == GVM_OK) {
    h.pending.push_back(Pending{0, nullptr, 0, 0, false, kMsgAttach});
    rc = wait_until(h, hdr, 10000000000ll, [&] { return h.finished.count(0) > 0; });
  }
  if (rc == GVM_OK) {
    rc = h.finished[0];
    h.finished.erase(0);
  }
  if (rc != GVM_OK) {
    h.data.close();
    s->pid.store(0);
    s->state.store(kSlotFree, std::memory_order_release);
    unmap_namespace();
    return rc;
  }
  h.attached = true;
  return GVM_OK;
}

int64_t rank_submit(int rank, int kernel_id, const void* in, void* out, uint64_t n, uint32_t flags) {
  if (rank < 0 || rank >= kMaxRanks) return fail(GVM_EINVAL, "rank %d out of range", rank);
  RankHandle& h = g_ranks[rank];
  std::lock_guard<std::mutex> lk(h.mu);
  if (!h.attached) return fail(GVM_ESTATE, "rank %d is not attached", rank);
  if (flags & ~(GVM_F_IN_RESIDENT | GVM_F_OUT_RESIDENT | GVM_F_NONBLOCK)) return fail(GVM_EINVAL, "unknown flags");
  Layout lay;
  if (!request_layout(kernel_id, n, &lay)) return fail(GVM_EINVAL, "bad kernel id %d or size %llu", kernel_id, (unsigned long long)n);
  CtlHeader* hdr = g_ns.hdr;
  uint8_t* base = static_cast<uint8_t*>(h.data.addr);
  const uint64_t size = h.data.bytes;
  auto inside = [&](const void* p, uint64_t bytes) {
    const uint8_t* q = static_cast<const uint8_t*>(p);
    return q >= base && q <= base + size && bytes <= static_cast<uint64_t>(base + size - q);
  };
  const bool in_res = flags & GVM_F_IN_RESIDENT;
  const bool out_res = flags & GVM_F_OUT_RESIDENT;
  if (!in_res && !in) return fail(GVM_EINVAL, "in is NULL");
  if (!out_res && !out) return fail(GVM_EINVAL, "out is NULL");
  const bool in_zero = !in_res && inside(in, lay.in_bytes);
  const bool out_zero = !out_res && inside(out, lay.out_bytes);
  const uint64_t need_in = (in_res || in_zero) ? 0 : align_up(lay.in_bytes, kAlign);
  const uint64_t need_out = (out_res || out_zero) ? 0 : align_up(lay.out_bytes, kAlign);
  if (need_in + need_out > size - h.user_region)
    return fail(GVM_ENOMEM, "request needs %llu bytes of shared memory, the rank has %llu",
                (unsigned long long)(need_in + need_out), (unsigned long long)(size - h.user_region));
  const uint64_t ticket = h.next_ticket;
  // room in the request ring (kRingCap - 1 outstanding keeps a response slot free)
  if (h.pending.size() >= kRingCap - 1) {
    if (flags & GVM_F_NONBLOCK) return fail(GVM_EAGAIN, "too many outstanding requests");
    int rc = wait_until(h, hdr, -1, [&] { return h.pending.size() < kRingCap - 1; });
    if (rc != GVM_OK) return rc;
  }
  uint64_t off = 0;
  while (!reserve(h, need_in + need_out, ticket, &off)) {
    if (flags & GVM_F_NONBLOCK) return fail(GVM_EAGAIN, "shared memory space busy");
    const size_t before = h.pending.size();
    if (before == 0) return fail(GVM_ENOMEM, "shared memory space too small");
    int rc = wait_until(h, hdr, -1, [&] { return h.pending.size() < before; });
    if (rc != GVM_OK) return rc;
  }
  Request m{};
  m.ticket = ticket;
  m.kernel_id = static_cast<uint32_t>(kernel_id);
  m.flags = flags & (GVM_F_IN_RESIDENT | GVM_F_OUT_RESIDENT);
  m.n = n;
  m.in_bytes = lay.in_bytes;
  m.out_bytes = lay.out_bytes;
  m.off_in = in_res ? 0 : (in_zero ? static_cast<uint64_t>(static_cast<const uint8_t*>(in) - base) : off);
  m.off_out = out_res ? 0 : (out_zero ? static_cast<uint64_t>(static_cast<uint8_t*>(out) - base) : off + need_in);
  if (need_in) rank_copy(base + m.off_in, in, lay.in_bytes, g_ns.hdr ? g_ns.hdr->nranks : 1);
  m.t_submit_ns = now_ns();
  int rc = push_message(h, hdr, m);
  if (rc != GVM_OK) {
    release(h, ticket);
    return rc;
  }
  h.next_ticket = ticket + 1;
  h.pending.push_back(Pending{ticket, out, m.off_out, lay.out_bytes, !out_res && !out_zero, static_cast<uint32_t>(kernel_id)});
  if (need_in + need_out == 0) release(h, ticket);
  return static_cast<int64_t>(ticket);
}

int rank_wait(int rank, int64_t ticket, int64_t timeout_ns, uint64_t* ts) {
  if (rank < 0 || rank >= kMaxRanks) return fail(GVM_EINVAL, "rank %d out of range", rank);
  RankHandle& h = g_ranks[rank];
  std::lock_guard<std::mutex> lk(h.mu);
  if (!h.attached) return fail(GVM_ESTATE, "rank %d is not attached", rank);
  CtlHeader* hdr = g_ns.hdr;
  if (ticket < 0) {
    int rc = wait_until(h, hdr, timeout_ns, [&] { return h.pending.empty(); });
    if (rc != GVM_OK) return rc;
    int worst = GVM_OK;
    for (auto& kv : h.finished)
      if (kv.second != GVM_OK && worst == GVM_OK) worst = kv.second;
    h.finished.clear();
    h.timing.clear();
    return worst;
  }
  const uint64_t t = static_cast<uint64_t>(ticket);
  drain(h);
  if (!h.finished.count(t)) {
    bool known = false;
    for (auto& p : h.pending) known |= (p.ticket == t);
    if (!known) return fail(GVM_EINVAL, "unknown ticket %lld", (long long)ticket);
  }
  int rc = wait_until(h, hdr, timeout_ns, [&] { return h.finished.count(t) > 0; });
  if (rc != GVM_OK) return rc;
  const int st = h.finished[t];
  h.finished.erase(t);
  auto it = h.timing.find(t);
  if (it != h.timing.end()) {
    if (ts) {
      ts[0] = it->second.t_submit_ns;
      ts[1] = it->second.t_admit_ns;
      ts[2] = it->second.t_launch_ns;
      ts[3] = it->second.t_device_ns;
      ts[4] = it->second.t_done_ns;
    }
    h.timing.erase(it);
  } else if (ts) {
    for (int i = 0; i < 5; ++i) ts[i] = 0;
  }
  return st;
}

int rank_wait_any(int rank, int64_t timeout_ns, int64_t* ticket_out, uint64_t* ts) {
  if (rank < 0 || rank >= kMaxRanks) return fail(GVM_EINVAL, "rank %d out of range", rank);
  RankHandle& h = g_ranks[rank];
  std::lock_guard<std::mutex> lk(h.mu);
  if (!h.attached) return fail(GVM_ESTATE, "rank %d is not attached", rank);
  drain(h);
  if (h.finished.empty() && h.pending.empty()) return fail(GVM_EINVAL, "nothing outstanding");
  int rc = wait_until(h, g_ns.hdr, timeout_ns, [&] { return !h.finished.empty(); });
  if (rc != GVM_OK) return rc;
  auto it = h.finished.begin();
  for (auto jt = h.finished.begin(); jt != h.finished.end(); ++jt)
    if (jt->first < it->first) it = jt;
  if (ticket_out) *ticket_out = static_cast<int64_t>(it->first);
  const int st = it->second;
  auto tt = h.timing.find(it->first);
  if (ts) {
    for (int i = 0; i < 5; ++i) ts[i] = 0;
    if (tt != h.timing.end()) {
      ts[0] = tt->second.t_submit_ns;
      ts[1] = tt->second.t_admit_ns;
      ts[2] = tt->second.t_launch_ns;
      ts[3] = tt->second.t_device_ns;
      ts[4] = tt->second.t_done_ns;
    }
  }
  if (tt != h.timing.end()) h.timing.erase(tt);
  h.finished.erase(it);
  return st;
}

int rank_detach(int rank) {
  if (rank < 0 || rank >= kMaxRanks) return fail(GVM_EINVAL, "rank %d out of range", rank);
  RankHandle& h = g_ranks[rank];
  std::lock_guard<std::mutex> lk(h.mu);
  if (!h.attached) return fail(GVM_ESTATE, "rank %d is not attached", rank);
  CtlHeader* hdr = g_ns.hdr;
  int rc = wait_until(h, hdr, -1, [&] { return h.pending.empty(); });
  if (rc == GVM_OK) {
    Request m{};
    m.kernel_id = kMsgDetach;
    m.ticket = h.next_ticket++;
    m.t_submit_ns = now_ns();
    const uint64_t t = m.ticket;
    rc = push_message(h, hdr, m);
    if (rc == GVM_OK) {
      h.pending.push_back(Pending{t, nullptr, 0, 0, false, kMsgDetach});
      rc = wait_until(h, hdr, 10000000000ll, [&] { return h.finished.count(t) > 0; });
    }
  }
  h.finished.clear();
  h.timing.clear();
  h.pending.clear();
  h.allocs.clear();
  h.data.close();
  if (!manager_gone(hdr)) {
    h.slot->pid.store(0, std::memory_order_relaxed);
    h.slot->state.store(kSlotFree, std::memory_order_release);
  }
  h.slot = nullptr;
  h.attached = false;
  unmap_namespace();
  return (rc == GVM_EDEAD) ? GVM_OK : rc;
}

void* rank_buffer(int rank, uint64_t bytes) {
  if (rank < 0 || rank >= kMaxRanks) {
    fail(GVM_EINVAL, "rank %d out of range", rank);
    return nullptr;
  }
  RankHandle& h = g_ranks[rank];
  std::lock_guard<std::mutex> lk(h.mu);
  if (!h.attached) {
    fail(GVM_ESTATE, "rank %d is not attached", rank);
    return nullptr;
  }
  const uint64_t want = align_up(bytes, 4096);
  if (want > h.data.bytes) {
    fail(GVM_ENOMEM, "rank space is %llu bytes", (unsigned long long)h.data.bytes);
    return nullptr;
  }
  if (want > h.user_region) {
    if (!h.allocs.empty()) {
      fail(GVM_ESTATE, "cannot grow the zero-copy region while requests hold the space");
      return nullptr;
    }
    h.user_region = want;
    h.head = want;
  }
  return h.data.addr;
}

int rank_detach_all() {
  int worst = GVM_OK;
  for (int r = 0; r < kMaxRanks; ++r) {
    bool att;
    {
      std::lock_guard<std::mutex> lk(g_ranks[r].mu);
      att = g_ranks[r].attached;
    }
    if (att) {
      int rc = rank_detach(r);
      if (rc != GVM_OK && worst == GVM_OK) worst = rc;
    }
  }
  return worst;
}

}  // namespace gvm
