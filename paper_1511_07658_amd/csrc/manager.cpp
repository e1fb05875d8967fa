#include "manager.hpp"

#include <dlfcn.h>
#include <immintrin.h>
#include <sched.h>
#include <pthread.h>
#include <time.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <future>
#include <new>

#include "common.hpp"

namespace gvm {

namespace {

// ROCTx ranges around the service loop's stages (GVM_ROCTX=1), so that a
// rocprofv3 marker trace shows the manager's host work beside the kernels:
// "gvm:drain" (rings), "gvm:complete" (completions and answers),
// "gvm:schedule" (barrier and admission), "gvm:launch" (enqueue).  The
// library is opened at run time; without the variable, or without the
// library, the ranges cost one branch.
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
  Roctx() {
    const char* e = getenv("GVM_ROCTX");
    if (!e || e[0] != '1') return;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!push || !pop) push = nullptr, pop = nullptr;
  }
};
const Roctx& roctx() {
  static const Roctx r;
  return r;
}
struct RoctxRange {
  explicit RoctxRange(const char* what) : on(roctx().push != nullptr) {
    if (on) roctx().push(what);
  }
  ~RoctxRange() {
    if (on) roctx().pop();
  }
  bool on;
};

}  // namespace

// ---------------------------------------------------------------- Arena

void Arena::init(uint64_t bytes) {
  free_.clear();
  total_ = bytes / 4096 * 4096;
  if (total_) free_[0] = total_;
  used_ = 0;
  peak_.store(0, std::memory_order_relaxed);
}

bool Arena::alloc(uint64_t bytes, uint64_t* off) {
  bytes = round(bytes);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const uint64_t rest = it->second - bytes;
      const uint64_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      if (used_ > peak_.load(std::memory_order_relaxed)) peak_.store(used_, std::memory_order_relaxed);
      return true;
    }
  }
  return false;
}

void Arena::release(uint64_t off, uint64_t bytes) {
  bytes = round(bytes);
  used_ -= bytes;
  auto it = free_.emplace(off, bytes).first;
  auto next = std::next(it);
  if (next != free_.end() && it->first + it->second == next->first) {
    it->second += next->second;
    free_.erase(next);
  }
  if (it != free_.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      free_.erase(it);
    }
  }
}

// ---------------------------------------------------------------- Manager

int Manager::init(const gvm_config& cfg_in) {
  if (started_) return fail(GVM_ESTATE, "a manager already runs in this process");
  if (cfg_in.size != sizeof(gvm_config)) return fail(GVM_EINVAL, "gvm_config.size mismatch");
  gvm_config cfg = cfg_in;
  if (cfg.nranks < 1 || cfg.nranks > static_cast<uint32_t>(kMaxRanks))
    return fail(GVM_EINVAL, "nranks must be in 1..%d", kMaxRanks);
  if (cfg.shm_bytes_per_rank < 4096) return fail(GVM_EINVAL, "shm_bytes_per_rank too small");
  if (cfg.hbm_budget_bytes < (1u << 20)) return fail(GVM_EINVAL, "hbm_budget_bytes must be >= 1 MiB");
  if (cfg.mode > GVM_MODE_SERVING || cfg.policy > GVM_POLICY_GROUPED || cfg.backend > GVM_BACKEND_LOOPBACK)
    return fail(GVM_EINVAL, "bad mode/policy/backend");
  // Graph replay captures a batch on the unmasked compute streams; the CU
  // partition launches on masked streams of its own, so the two do not mix.
  if (cfg.use_graphs && cfg.latency_cus) return fail(GVM_EINVAL, "use_graphs and latency_cus cannot be combined");
  if (cfg.latency_cus && (cfg.mode != GVM_MODE_SERVING || cfg.latency_cus % 32 || cfg.latency_cus >= 256))
    return fail(GVM_EINVAL, "latency_cus must be 0, or in serving mode a multiple of 32 below 256");
  cfg.shm_bytes_per_rank = (cfg.shm_bytes_per_rank + 4095) / 4096 * 4096;
  if (const char* e = getenv("GVM_RANK_DEPTH")) rank_depth_ = (e[0] == '1') ? 1 : kRankDepth;
  if (cfg.max_inflight == 0) cfg.max_inflight = cfg.nranks * static_cast<uint32_t>(rank_depth_);
  spin_ns_ = spin_env_ns("GVM_MANAGER_SPIN_US", 200);
  // Piece size of the piecewise copies.  Batch mode moves a whole step's
  // inputs and results in two FIFO streams: larger pieces carry less fixed
  // cost per byte (16 MiB: 2-5 % shorter copy-inclusive steps than 8 MiB,
  // 32 MiB about 1 % shorter again).
  // Serving mode interleaves many small requests with large ones, where a
  // piece is the unit a small request waits behind (16 MiB doubled p50 at
  // 2000 requests/s).
  set_piece_bytes(cfg.mode == GVM_MODE_BATCH ? (32ull << 20) : (8ull << 20));
  cfg.name[GVM_NAME_MAX - 1] = 0;
  cfg_ = cfg;
  ns_ = cfg.name[0] ? std::string(cfg.name) : default_namespace();
  if (ns_.find('/') != std::string::npos) return fail(GVM_EINVAL, "namespace must not contain '/'");

  int rc = ctl_seg_.create(ctl_object_name(ns_), ctl_bytes(cfg.nranks));
  if (rc != GVM_OK) return rc;
  ctl_ = new (ctl_seg_.addr) CtlHeader();
  ctl_->magic = kMagic;
  ctl_->version = kVersion;
  ctl_->nranks = cfg.nranks;
  ctl_->shm_bytes_per_rank = cfg.shm_bytes_per_rank;
  ctl_->slot_stride = ctl_slot_stride();
  ctl_->state.store(kStarting);
  ctl_->manager_pid.store(getpid());
  ctl_->generation.store(static_cast<uint32_t>(now_ns() & 0xffffffffu));
  ctl_->bell.store(0);
  ctl_->manager_sleeping.store(0);
  ctl_->group_bell.store(0);
  ctl_->cfg = cfg;
  for (uint32_t r = 0; r < cfg.nranks; ++r) {
    RankSlot* s = new (ctl_slot(ctl_, r)) RankSlot();
    s->state.store(kSlotFree);
    s->pid.store(0);
    s->epoch.store(0);
    s->resp_bell.store(0);
    s->rank_sleeping.store(0);
    s->req.reset();
    s->resp.reset();
  }
  data_.clear();
  for (uint32_t r = 0; r < cfg.nranks; ++r) {
    auto seg = std::make_unique<Segment>();
    rc = seg->create(data_object_name(ns_, r), cfg.shm_bytes_per_rank);
    if (rc != GVM_OK) {
      data_.clear();
      ctl_seg_.close();
      ctl_ = nullptr;
      return rc;
    }
    data_.push_back(std::move(seg));
  }
  ranks_.assign(cfg.nranks, RankRt{});
  arena_.init(cfg.hbm_budget_bytes);
  copy_.start(cfg.copy_threads ? static_cast<int>(cfg.copy_threads) : 4);
  dev_ = (cfg.backend == GVM_BACKEND_LOOPBACK) ? make_loopback_device() : make_hip_device();

  // The service thread opens the device itself so that every HIP call of the
  // manager is made from one thread.
  stop_.store(false);
  std::promise<int> ready;
  std::future<int> fut = ready.get_future();
  thread_ = std::thread([this, &ready] { service(&ready); });
  rc = fut.get();
  if (rc != GVM_OK) {
    thread_.join();
    copy_.stop();
    fail(rc, "%s", open_error_.c_str());
    dev_.reset();
    data_.clear();
    ctl_seg_.close();
    ctl_ = nullptr;
    return rc;
  }
  started_ = true;
  stats_t0_ns_ = now_ns();
  stats_cpu0_ns_ = service_cpu_ns();
  return GVM_OK;
}

void Manager::service(std::promise<int>* ready) {
  int rc = dev_->open(cfg_);
  if (rc != GVM_OK) {
    open_error_ = last_error_text();
    dev_->close();
    ready->set_value(rc);
    return;
  }
  ctl_->heartbeat_ns.store(now_ns());
  ctl_->state.store(kReady, std::memory_order_release);
  ready->set_value(GVM_OK);

  uint32_t spins = 0;
  uint64_t idle_since = 0;
  while (!stop_.load(std::memory_order_acquire)) {
    ctl_->heartbeat_ns.store(now_ns(), std::memory_order_relaxed);
    if (reset_pending_.exchange(false)) {
      dev_->flush_retired();  // work before the reset stays out of the counters
      dev_->reset_stats();
      arena_.reset_peak();
    }
    if (flush_req_.exchange(false)) {
      flush_deferred();
      {
        std::lock_guard<std::mutex> lk(flush_mu_);
        ++flush_done_;
      }
      flush_cv_.notify_all();
    }
    const uint64_t t_it = now_ns();
    bool progress;
    bool done;
    {
      RoctxRange rr("gvm:drain");
      progress = drain_rings();
    }
    {
      RoctxRange rr("gvm:complete");
      done = complete_jobs();
    }
    wake_group();
    const uint64_t t_done = now_ns();
    progress |= done;
    check_liveness();
    bool launched;
    {
      RoctxRange rr("gvm:schedule");
      progress |= schedule();
    }
    {
      RoctxRange rr("gvm:launch");
      launched = launch_ready();
    }
    progress |= launched;
    wake_group();  // answers given while scheduling or launching
    if (progress) {
      // time of service iterations that retired or launched work (the ring
      // is not drained while they run)
      if (done || launched) {
        const uint64_t t_end = now_ns();
        std::lock_guard<std::mutex> lk(stats_mu_);
        if (iter_us_.size() < (1u << 20)) {
          iter_us_.push_back((t_end - t_it) * 1e-3);
          iter_done_us_.push_back((t_done - t_it) * 1e-3);
        }
      }
      spins = 0;
      idle_since = 0;
      continue;
    }
    if (inflight_ > 0 && !early_idle()) {
      // device work outstanding: retire finished batches meanwhile, then
      // poll its events, yielding the core politely
      flush_deferred();
      if (++spins < 64) _mm_pause(); else sched_yield();
      idle_since = 0;
      continue;
    }
    // just went idle: keep polling the rings for a short while, so that the
    // next request of a synchronous SPMD step is seen without a futex wake-up
    if (idle_since == 0) idle_since = now_ns();
    if (now_ns() - idle_since < spin_ns_) {
      // (finished batches are retired while the device works, or before the
      // sleep below, not here: a synchronous rank's next request is due now)
      // yield now and then, for a rank that shares this core
      if (++spins % 64 == 0) sched_yield(); else _mm_pause();
      continue;
    }
    // idle: retire what finished, then sleep on the doorbell until a rank
    // rings it (or a deadline)
    flush_deferred();
    int64_t timeout = 2000000;  // 2 ms: liveness checks and batch windows
    const uint32_t v = ctl_->bell.load(std::memory_order_acquire);
    ctl_->manager_sleeping.store(1, std::memory_order_seq_cst);
    std::atomic_thread_fence(std::memory_order_seq_cst);
    if (!any_request_waiting()) {
      if (cfg_.mode == GVM_MODE_BATCH && cfg_.batch_window_us) {
        bool waiting = !early_.empty();
        for (const auto& rt : ranks_) waiting |= !rt.queue.empty();
        if (waiting) timeout = std::min<int64_t>(timeout, int64_t(cfg_.batch_window_us) * 1000 / 4 + 1000);
      }
      futex_wait(&ctl_->bell, v, timeout);
    }
    ctl_->manager_sleeping.store(0, std::memory_order_relaxed);
    spins = 0;
    idle_since = 0;
  }

  // Shutdown: let device work finish (requests admitted early run as a
  // last batch), answer what is still queued.
  staged_.insert(staged_.end(), early_.begin(), early_.end());
  early_.clear();
  while (inflight_ > 0) {
    launch_ready();
    complete_jobs();
    if (inflight_ > 0) sched_yield();
  }
  copy_.stop();
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    drain_rings();
    auto& rt = ranks_[r];
    while (!rt.queue.empty()) {
      const Queued q = rt.queue.front();
      rt.queue.pop_front();
      respond(r, q.req.ticket, q.req.kernel_id, GVM_ECANCELED, nullptr, q.req.t_submit_ns);
    }
  }
  ctl_->state.store(kStopping, std::memory_order_release);
  dev_->close();
  ctl_->state.store(kStopped, std::memory_order_release);
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    RankSlot* s = ctl_slot(ctl_, r);
    s->resp_bell.fetch_add(1);
    futex_wake_all(&s->resp_bell);
  }
  ctl_->group_bell.fetch_add(1);
  futex_wake_all(&ctl_->group_bell);
}

// One wake-up call for every rank that fell asleep on the group doorbell
// since the last call (respond() only marks them).
void Manager::wake_group() {
  if (!group_wake_) return;
  group_wake_ = false;
  ctl_->group_bell.fetch_add(1, std::memory_order_seq_cst);
  futex_wake_all(&ctl_->group_bell);
}

bool Manager::any_request_waiting() const {
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    RankSlot* s = ctl_slot(ctl_, r);
    if (s->state.load(std::memory_order_acquire) != kSlotFree && !s->req.empty()) return true;
  }
  return false;
}

bool Manager::drain_rings() {
  bool any = false;
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    RankSlot* s = ctl_slot(ctl_, r);
    if (s->state.load(std::memory_order_acquire) == kSlotFree) continue;
    Request m;
    while (s->req.pop(&m)) {
      on_message(static_cast<int>(r), m);
      any = true;
    }
  }
  return any;
}

void Manager::on_message(int r, const Request& m) {
  RankSlot* s = ctl_slot(ctl_, r);
  RankRt& rt = ranks_[r];
  if (m.kernel_id == kMsgAttach) {
    if (rt.attached) release_slot(r);
    rt = RankRt{};
    rt.attached = true;
    rt.pid = s->pid.load(std::memory_order_acquire);
    rt.last_use_ns = now_ns();
    s->state.store(kSlotAttached, std::memory_order_release);
    respond(r, m.ticket, m.kernel_id, GVM_OK, nullptr, m.t_submit_ns);
    return;
  }
  if (!rt.attached) return;  // stray message of a slot that is not attached
  if (m.kernel_id == kMsgDetach) {
    rt.detach_pending = true;
    rt.detach_ticket = m.ticket;
    return;
  }
  Queued q{seq_++, now_ns(), GVM_OK, m};
  if (m.t_submit_ns && q.t_arrive_ns >= m.t_submit_ns) {
    std::lock_guard<std::mutex> lk(stats_mu_);
    if (ring_us_.size() < (1u << 20)) ring_us_.push_back((q.t_arrive_ns - m.t_submit_ns) * 1e-3);
  }
  Layout lay;
  const uint64_t space = cfg_.shm_bytes_per_rank;
  if (!request_layout(static_cast<int>(m.kernel_id), m.n, &lay) || lay.in_bytes != m.in_bytes ||
      lay.out_bytes != m.out_bytes) {
    q.status = GVM_EINVAL;
  } else if (slot_bytes(lay) > arena_.total()) {
    q.status = GVM_ENOMEM;
  } else if (!(m.flags & GVM_F_IN_RESIDENT) && (m.off_in > space || lay.in_bytes > space - m.off_in)) {
    q.status = GVM_EINVAL;
  } else if (!(m.flags & GVM_F_OUT_RESIDENT) && (m.off_out > space || lay.out_bytes > space - m.off_out)) {
    q.status = GVM_EINVAL;
  } else if (slot_out_offset(lay) + lay.out_bytes > align_up((cfg_.staging_bytes ? cfg_.staging_bytes : space) + 2 * kAlign, 4096)) {
    q.status = GVM_ENOMEM;  // the pinned staging mirrors the slot's input and output
  }
  rt.queue.push_back(q);
}

void Manager::respond(int r, uint64_t ticket, uint32_t kernel_id, int status, const Job* j, uint64_t t_submit) {
  RankSlot* s = ctl_slot(ctl_, r);
  Response resp{};
  resp.ticket = ticket;
  resp.status = status;
  resp.kernel_id = kernel_id;
  resp.t_submit_ns = t_submit;
  if (j) {
    resp.t_admit_ns = j->t_admit_ns;
    resp.t_launch_ns = j->t_launch_ns;
    resp.t_device_ns = j->t_device_ns;
  }
  resp.t_done_ns = now_ns();
  // The rank keeps at most kRingCap - 1 requests outstanding, so there is
  // always room for a response; spin briefly if the rank is slow to drain.
  int tries = 0;
  while (!s->resp.push(resp)) {
    if (++tries > 1000000) return;  // rank is gone; drop
    sched_yield();
  }
  std::atomic_thread_fence(std::memory_order_seq_cst);
  s->resp_bell.fetch_add(1, std::memory_order_seq_cst);
  const uint32_t sleep = s->rank_sleeping.load(std::memory_order_seq_cst);
  if (sleep == kSleepOwnBell) futex_wake_all(&s->resp_bell);
  else if (sleep == kSleepGroupBell) group_wake_ = true;  // woken with the rest by wake_group()
  if (kernel_id >= GVM_K_VECADD && kernel_id <= GVM_K_EP) {
    std::lock_guard<std::mutex> lk(stats_mu_);
    const TraceRec tr{r, kernel_id, status, 0, j ? j->req.n : 0, ticket, t_submit, resp.t_admit_ns,
                      resp.t_launch_ns, resp.t_device_ns, resp.t_done_ns};
    if (trace_.size() < kTraceMax) {
      trace_.push_back(tr);
    } else {
      trace_[trace_next_] = tr;
      trace_next_ = (trace_next_ + 1) % kTraceMax;
    }
    ++n_traced_;
    if (status == GVM_OK) {
      ++n_done_;
      auto& v = lat_us_[kernel_id];
      if (v.size() < (1u << 20)) v.push_back((resp.t_done_ns - t_submit) * 1e-3);
      if (j && wait_us_.size() < (1u << 20)) wait_us_.push_back((j->t_admit_ns - t_submit) * 1e-3);
    } else {
      ++n_err_;
    }
  }
}

void Manager::release_slot(int r) {
  RankRt& rt = ranks_[r];
  if (rt.has_slot) arena_.release(rt.slot_off, rt.slot_size);
  rt.has_slot = false;
  rt.slot_off = rt.slot_size = 0;
  rt.res_valid = false;
}

// A rank process died: drop its queue, free its memory once its device work
// is done, and free its slot for a new attach.
void Manager::reap_rank(int r) {
  RankRt& rt = ranks_[r];
  rt.queue.clear();
  if (!rt.running.empty()) return;  // finish the device work first; complete_jobs calls back
  release_slot(r);
  rt = RankRt{};
  RankSlot* s = ctl_slot(ctl_, r);
  Request m;
  while (s->req.pop(&m)) {
  }
  s->pid.store(0, std::memory_order_relaxed);
  s->state.store(kSlotFree, std::memory_order_release);
}

void Manager::check_liveness() {
  const uint64_t now = now_ns();
  if (now - last_liveness_ns_ < 20000000) return;  // every 20 ms
  last_liveness_ns_ = now;
  const int32_t self = getpid();
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    RankSlot* s = ctl_slot(ctl_, r);
    RankRt& rt = ranks_[r];
    const uint32_t st = s->state.load(std::memory_order_acquire);
    if (st == kSlotFree) continue;
    const int32_t pid = rt.attached ? rt.pid : s->pid.load(std::memory_order_acquire);
    if (pid == 0 || pid == self) continue;
    if (!pid_alive(pid)) reap_rank(static_cast<int>(r));
  }
}

// Device completions and host copy-outs, per rank (up to kRankDepth jobs in
// flight each).
bool Manager::complete_jobs() {
  bool any = false;
  dev_->begin_poll();
  // 1. device work that finished: start the result's copy-out
  std::vector<Job*> device_done;
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    for (Job* j : ranks_[r].running) {
      if (j->stage != kStageDevice) continue;
      const uint64_t out_off = slot_out_offset(j->lay);
      if (j->out_pieces && j->status == GVM_OK) {
        // hand each output piece to the host copy as soon as it is staged
        const int n = dev_->out_pieces_done(j);
        if (n < 0) {
          j->status = n;
        } else {
          for (; j->out_taken < static_cast<uint32_t>(n); ++j->out_taken) {
            const uint64_t off = static_cast<uint64_t>(j->out_taken) * piece_bytes();
            copy_.submit(j->shm + j->req.off_out + off, j->pin + out_off + off,
                         std::min<uint64_t>(piece_bytes(), j->lay.out_bytes - off), &j->copies, j->small);
            any = true;
          }
          if (j->out_taken < j->out_pieces) continue;
        }
      }
      if (dev_->query(j) == 0) continue;
      device_done.push_back(j);
      any = true;
      if (j->status == GVM_OK && j->copy_out && !j->out_pieces)
        copy_.submit(j->shm + j->req.off_out, j->pin + out_off, j->lay.out_bytes, &j->copies, j->small);
      j->stage = kStageCopyOut;
    }
  }
  // 2. answer every job whose result is in place, before any bookkeeping
  std::vector<Job*> answered;
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    RankRt& rt = ranks_[r];
    for (Job* j : rt.running) {
      if (j->stage != kStageCopyOut || j->copies.load(std::memory_order_acquire) != 0) continue;
      if (rt.attached) respond(static_cast<int>(r), j->req.ticket, j->req.kernel_id, j->status, j, j->req.t_submit_ns);
      answered.push_back(j);
    }
  }
  // 3. release the device bookkeeping (event timings of a retired batch)
  for (Job* j : device_done) dev_->finish(j);
  // 4. retire the answered jobs
  for (Job* j : answered) {
    const int r = j->rank;
    RankRt& rt = ranks_[r];
    const bool alive = rt.attached;
    if (j->status != GVM_OK && !j->extra_slot) rt.res_valid = false;
    rt.running.erase(std::find(rt.running.begin(), rt.running.end(), j));
    if (j->extra_slot) {
      if (rt.running.empty() && j->req.ticket == rt.last_ticket) {
        // the rank's latest request finished last: its slot becomes the
        // rank's resident slot, as if it had run alone
        release_slot(r);
        rt.has_slot = true;
        rt.slot_off = j->extra_off;
        rt.slot_size = j->extra_size;
        rt.res_valid = j->status == GVM_OK;
        rt.res_kernel = j->req.kernel_id;
        rt.res_n = j->req.n;
      } else {
        arena_.release(j->extra_off, j->extra_size);
      }
    }
    rt.last_use_ns = now_ns();
    delete j;
    --inflight_;
    any = true;
    if (!alive) reap_rank(r);  // a dead rank process is found by check_liveness()
  }
  if (cfg_.mode == GVM_MODE_BATCH && batch_open_ && inflight_ == early_.size()) batch_open_ = false;
  return any;
}

void Manager::flush_deferred() {
  if (!dev_->flush_retired()) return;
  std::lock_guard<std::mutex> lk(stats_mu_);
  const KernelStats* ks = dev_->kernel_stats();
  for (int k = 0; k < kNumKernelIds; ++k) kstats_[k] = ks[k];
  peak_bytes_ = std::max(peak_bytes_, arena_.peak());
  if (cfg_.batch_timing) timing_json_ = dev_->timing_json();
}

// Move an admitted job's copy-in along: each input piece goes to the device
// as soon as it is staged.  True once the job is ready to launch (its whole
// input staged, and sent when it goes in pieces).
bool Manager::forward_pieces(Job* j) {
  if (j->stage == kStageCopyIn) {
    if (j->pieces) {
      while (j->in_sent < j->in_pieces && j->in_pending[j->in_sent].load(std::memory_order_acquire) == 0) {
        const uint64_t off = static_cast<uint64_t>(j->in_sent) * piece_bytes();
        const int rc = dev_->stream_in(j, off, std::min<uint64_t>(piece_bytes(), j->lay.in_bytes - off));
        if (rc != GVM_OK && j->status == GVM_OK) j->status = rc;
        ++j->in_sent;
      }
      if (j->in_sent == j->in_pieces) j->stage = kStageReady;
    } else if (j->copies.load(std::memory_order_acquire) == 0) {
      j->stage = kStageReady;
    }
  }
  return j->stage == kStageReady;
}

// Early copy-in holds nothing the service loop must poll for: the batch has
// retired and every early job is ready (its input staged and sent), so the
// loop may sleep until the remaining ranks ring.
bool Manager::early_idle() const {
  if (early_.empty() || inflight_ != early_.size()) return false;
  for (const Job* j : early_)
    if (j->stage != kStageReady) return false;
  return true;
}

// Launch what is ready, then move the early requests' copy-in along (after
// the launch, so that a grouped batch's wait for the copy FIFO covers its
// own inputs only).
bool Manager::launch_ready() {
  const bool launched = launch_staged();
  for (Job* j : early_) forward_pieces(j);
  return launched;
}

// Launch admitted jobs whose inputs have reached the pinned staging.  A
// batch (batch mode) goes to the device as a whole once every input is in;
// in serving mode every ready job goes as soon as its copy-in lands.
bool Manager::launch_staged() {
  if (staged_.empty()) return false;
  bool all = true;
  for (Job* j : staged_) all &= forward_pieces(j);
  // A batch of kernels that run as one grouped launch waits for all of its
  // inputs; per-rank launches (PS-2, what AUTO picks when large data moves) start
  // as soon as each input has landed, overlapping the others' copies.  With
  // batch_timing a batch is enqueued as a whole (one device-phase span).
  bool incremental = cfg_.mode == GVM_MODE_SERVING || cfg_.policy == GVM_POLICY_PS2;
  if (cfg_.policy == GVM_POLICY_AUTO)
    for (const Job* j : staged_) incremental |= (j->copy_in || j->copy_out) && !j->local;  // as resolve_policy
  if (cfg_.mode == GVM_MODE_BATCH && cfg_.batch_timing) incremental = false;
  std::vector<Job*> ready;
  if (!incremental) {
    if (!all) return false;
    ready.swap(staged_);
  } else {
    // Batch mode: at most kLaunchChunk per call.  Enqueueing a request's
    // per-rank chain (waits, kernel, output pieces with an event each) takes
    // the host about 45 us, so a 32-rank batch held the service loop for
    // 1.5 ms while the first results were already back; between chunks the
    // loop answers them, and those ranks' next inputs start (early copy-in).
    const size_t cap = cfg_.mode == GVM_MODE_BATCH ? kLaunchChunk : staged_.size();
    std::vector<Job*> keep;
    for (Job* j : staged_) (j->stage == kStageReady && ready.size() < cap ? ready : keep).push_back(j);
    staged_.swap(keep);
    if (ready.empty()) return false;
  }
  const int policy = resolve_policy(ready);
  for (Job* j : ready) j->stage = kStageDevice;
  if (cfg_.latency_cus == 0) {
    dev_->launch(ready, policy);
  } else {
    // spatial partition: the latency class and the rest launch separately,
    // each on its own CU-masked stream
    std::vector<Job*> part[2];
    for (Job* j : ready) {
      j->part = estimate_device_us(static_cast<int>(j->req.kernel_id), j->req.n) <= kLatencyClassUs ? 0 : 1;
      part[j->part].push_back(j);
    }
    for (auto& v : part)
      if (!v.empty()) dev_->launch(v, policy);
  }
  std::lock_guard<std::mutex> lk(stats_mu_);
  ++n_batches_;
  return true;
}

Manager::Admit Manager::admit(int r, std::vector<Job*>& jobs) {
  RankRt& rt = ranks_[r];
  // a copy: the queue entry is popped below, before the last reads of the request
  const Request m = rt.queue.front().req;
  Layout lay;
  request_layout(static_cast<int>(m.kernel_id), m.n, &lay);
  const uint64_t need = slot_bytes(lay);
  const bool second = !rt.running.empty();  // pipelined behind the rank's request in flight
  uint64_t pin_off = 0;
  if (second) {
    // rank_can_take() let only plain requests of a serving rank through; the
    // staging region goes after (or before) the first request's, if it fits
    const Job* first = rt.running.front();
    const uint64_t staging = cfg_.staging_bytes ? cfg_.staging_bytes : cfg_.shm_bytes_per_rank;
    const uint64_t len = Arena::round(need);
    if (len <= first->pin_off) {
      pin_off = 0;
    } else if (Arena::round(first->pin_off + first->pin_len) + len <= staging) {
      pin_off = Arena::round(first->pin_off + first->pin_len);
    } else {
      return kNotNow;  // both do not fit the staging: wait for the first
    }
  }
  if (m.flags & GVM_F_IN_RESIDENT) {
    if (!(rt.res_valid && rt.res_kernel == m.kernel_id && rt.res_n == m.n && rt.has_slot)) {
      respond(r, m.ticket, m.kernel_id, fail(GVM_ESTATE, "no resident input for this request"), nullptr, m.t_submit_ns);
      rt.queue.pop_front();
      return kRejected;
    }
  }
  uint64_t extra_off = 0;
  auto alloc_evicting = [&](uint64_t* off) {
    while (!arena_.alloc(need, off)) {
      // evict the least recently used idle rank's resident buffer
      int victim = -1;
      for (uint32_t v = 0; v < cfg_.nranks; ++v) {
        const RankRt& o = ranks_[v];
        if (static_cast<int>(v) == r || !o.has_slot || !o.running.empty()) continue;
        if (victim < 0 || o.last_use_ns < ranks_[victim].last_use_ns) victim = static_cast<int>(v);
      }
      if (victim < 0) return false;
      release_slot(victim);
    }
    return true;
  };
  if (second) {
    // a device slot of its own, freed when the request is answered
    if (!alloc_evicting(&extra_off)) return kWait;
  } else if (!(rt.has_slot && rt.slot_size >= need)) {
    release_slot(r);
    uint64_t off = 0;
    if (!alloc_evicting(&off)) return kWait;
    rt.has_slot = true;
    rt.slot_off = off;
    rt.slot_size = Arena::round(need);
  }
  uint8_t* pin = nullptr;
  const bool copy_in = !(m.flags & GVM_F_IN_RESIDENT);
  const bool copy_out = !(m.flags & GVM_F_OUT_RESIDENT);
  if (copy_in || copy_out) {
    pin = dev_->staging(r);
    if (!pin) {
      if (second) arena_.release(extra_off, Arena::round(need));
      respond(r, m.ticket, m.kernel_id, GVM_EDEVICE, nullptr, m.t_submit_ns);
      rt.queue.pop_front();
      return kRejected;
    }
    pin += pin_off;
  }
  Job* j = new Job;
  j->rank = r;
  j->req = m;
  j->lay = lay;
  j->shm = static_cast<uint8_t*>(data_[r]->addr);
  j->slot = dev_->arena() + (second ? extra_off : rt.slot_off);
  j->extra_slot = second;
  j->extra_off = extra_off;
  j->extra_size = second ? Arena::round(need) : 0;
  j->pin_off = pin_off;
  j->pin_len = Arena::round(need);
  j->pin = pin;
  j->copy_in = copy_in;
  j->copy_out = copy_out;
  j->t_admit_ns = now_ns();
  // small copies stay with the kernel; whole copies where a batch's device
  // phase is timed as one span; pieces otherwise (each piece is enqueued when
  // it lands, outside any graph)
  j->local = (copy_in ? lay.in_bytes : 0) + (copy_out ? lay.out_bytes : 0) <= kLocalCopyBytes;
  // serving: small requests take the copy threads first
  j->small = cfg_.mode == GVM_MODE_SERVING && cfg_.small_request_bytes &&
             lay.in_bytes + lay.out_bytes <= cfg_.small_request_bytes;
  j->pieces = !j->local && !(cfg_.batch_timing && cfg_.mode == GVM_MODE_BATCH);
  if (j->pieces && copy_out) j->out_pieces = piece_count(lay.out_bytes);
  if (copy_in) {
    j->stage = kStageCopyIn;
    if (j->pieces) {
      j->in_pieces = piece_count(lay.in_bytes);
      j->in_pending.reset(new std::atomic<int>[j->in_pieces]());
      for (uint32_t i = 0; i < j->in_pieces; ++i) {
        const uint64_t off = static_cast<uint64_t>(i) * piece_bytes();
        const uint64_t len = std::min<uint64_t>(piece_bytes(), lay.in_bytes - off);
        j->in_pending[i].store(0, std::memory_order_relaxed);
        copy_.submit(j->pin + off, j->shm + m.off_in + off, len, &j->in_pending[i], j->small);
      }
    } else {
      copy_.submit(j->pin, j->shm + m.off_in, lay.in_bytes, &j->copies, j->small);
    }
  } else {
    j->stage = kStageReady;
  }
  rt.queue.pop_front();
  rt.running.push_back(j);
  rt.last_ticket = m.ticket;
  if (second) {
    // the rank's slot keeps the first request's input: nothing of the latest
    // request stays resident
    rt.res_valid = false;
  } else {
    rt.res_valid = true;
    rt.res_kernel = m.kernel_id;
    rt.res_n = m.n;
  }
  ++inflight_;
  jobs.push_back(j);
  return kAdmitted;
}

int Manager::resolve_policy(const std::vector<Job*>& jobs) const {
  if (cfg_.policy != GVM_POLICY_AUTO) return static_cast<int>(cfg_.policy);
  // Resident requests (no copies) are pure kernel work: one grouped launch.
  // With copies every kernel here is I/O-intensive on this GPU by the test of
  // Section 4.2.3 (PCIe time exceeds kernel time), so the paper's rule gives
  // PS-2, which overlaps each rank's copies with the others' kernels.  Small
  // copies (at most kLocalCopyBytes per request, kept on the kernel's own
  // stream) are the exception: there a cross-queue dependency costs more
  // than the copies, and one grouped launch is faster (measured 0.48 ms
  // grouped against 0.68 ms PS-2 for 8 x vecadd 64K, 0.49 against 0.68 for
  // 8 x SGEMM 256).
  bool large = false;
  for (const Job* j : jobs) large |= (j->copy_in || j->copy_out) && !j->local;
  return large ? GVM_POLICY_PS2 : GVM_POLICY_GROUPED;
}

bool Manager::rank_can_take(const RankRt& rt) const {
  if (rt.running.empty()) return true;
  if (cfg_.mode != GVM_MODE_SERVING || rt.running.size() >= rank_depth_) return false;
  const Queued& q = rt.queue.front();
  // error heads and requests that use the rank's resident slot wait for it
  return q.status == GVM_OK && !(q.req.flags & (GVM_F_IN_RESIDENT | GVM_F_OUT_RESIDENT));
}

bool Manager::schedule() {
  bool any = false;
  // Heads that were invalid on arrival are answered in order.
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    RankRt& rt = ranks_[r];
    while (rt.running.empty() && !rt.queue.empty() && rt.queue.front().status != GVM_OK) {
      const Queued q = rt.queue.front();
      rt.queue.pop_front();
      respond(static_cast<int>(r), q.req.ticket, q.req.kernel_id, q.status, nullptr, q.req.t_submit_ns);
      any = true;
    }
    if (rt.detach_pending && rt.queue.empty() && rt.running.empty()) {
      release_slot(static_cast<int>(r));
      const uint64_t t = rt.detach_ticket;
      rt = RankRt{};
      respond(static_cast<int>(r), t, kMsgDetach, GVM_OK, nullptr, now_ns());
      any = true;
    }
  }

  // Candidate heads in global arrival order.
  std::vector<std::pair<uint64_t, int>> heads;
  size_t live = 0;
  uint64_t oldest = UINT64_MAX, newest = 0;
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    const RankRt& rt = ranks_[r];
    if (!rt.attached) continue;
    ++live;
    if (rt.queue.empty() || !rank_can_take(rt)) continue;
    heads.emplace_back(rt.queue.front().seq, static_cast<int>(r));
    oldest = std::min(oldest, rt.queue.front().t_arrive_ns);
    newest = std::max(newest, rt.queue.front().t_arrive_ns);
  }
  if (heads.empty() && early_.empty()) return any;
  std::sort(heads.begin(), heads.end());

  std::vector<Job*> jobs;
  if (cfg_.mode == GVM_MODE_BATCH) {
    if (batch_open_) {
      // Early copy-in: once every input of the running batch is on its way
      // (its jobs still in staged_ wait only for their launch), a rank whose
      // request has been answered moves its next input now, while the
      // batch's results leave over the link in the other direction.  The
      // request still waits for the barrier below before its kernel runs.
      const bool early = cfg_.early_copy_in && !cfg_.batch_timing && !cfg_.use_graphs;
      bool inputs_sent = true;  // every input of the running batch is on the copy FIFO
      for (const Job* j : staged_) inputs_sent &= j->stage == kStageReady;
      if (early && inputs_sent) {
        for (auto& h : heads) {
          const Queued& q = ranks_[h.second].queue.front();
          if (q.status != GVM_OK || (q.req.flags & GVM_F_IN_RESIDENT)) continue;
          const uint64_t t = q.t_arrive_ns;
          std::vector<Job*> got;
          if (admit(h.second, got) == kRejected) any = true;
          for (Job* j : got) {
            if (early_.empty() || t < early_oldest_ns_) early_oldest_ns_ = t;
            early_newest_ns_ = early_.empty() ? t : std::max(early_newest_ns_, t);
            early_.push_back(j);
            any = true;
          }
        }
      }
      return any;
    }
    // Request barrier (Section 5): run when every attached rank has a
    // request (queued, or admitted early), or when the window since the
    // oldest one has passed.
    if (!early_.empty()) {
      oldest = std::min(oldest, early_oldest_ns_);
      newest = std::max(newest, early_newest_ns_);
    }
    const bool all = heads.size() + early_.size() >= live;
    const bool expired = now_ns() - oldest >= static_cast<uint64_t>(cfg_.batch_window_us) * 1000ull;
    if (!all && !expired) return any;
    {
      std::lock_guard<std::mutex> lk(stats_mu_);
      if (batch_lag_us_.size() < (1u << 20)) batch_lag_us_.push_back((now_ns() - newest) * 1e-3);
    }
    // Order of the batch's copies: the requests move host -> device, then
    // device -> host, each direction one FIFO (the two copy engines of the
    // execution model, Section 4.2.3), a two-stage flow shop.  Every kernel
    // here sends back less than it receives (half for vector add and SGEMM,
    // two thirds for Black-Scholes), and for such jobs the shortest schedule
    // takes them by decreasing result size (Johnson's rule): the link's
    // last transfer after the final input is then the smallest result.
    auto out_bytes = [&](int r) {
      Layout l;
      const Request& q = ranks_[r].queue.front().req;
      if (!request_layout(static_cast<int>(q.kernel_id), q.n, &l)) return uint64_t(0);
      return (q.flags & GVM_F_OUT_RESIDENT) ? uint64_t(0) : l.out_bytes;
    };
    std::stable_sort(heads.begin(), heads.end(), [&](const std::pair<uint64_t, int>& x, const std::pair<uint64_t, int>& y) {
      return out_bytes(x.second) > out_bytes(y.second);
    });
    for (auto& h : heads) {
      Admit a = admit(h.second, jobs);
      if (a == kRejected) any = true;
    }
    // the early requests lead: their copies started first
    jobs.insert(jobs.begin(), early_.begin(), early_.end());
    early_.clear();
  } else {
    for (auto& h : heads) {
      if (inflight_ >= cfg_.max_inflight) break;
      Admit a = admit(h.second, jobs);
      if (a == kWait) break;  // first-come first-served: nobody overtakes a waiting head
      if (a == kRejected) any = true;
      // kNotNow: a second request of a rank that must wait for the rank's
      // first; it holds up no other rank
    }
  }
  if (jobs.empty()) return any;
  staged_.insert(staged_.end(), jobs.begin(), jobs.end());
  if (cfg_.mode == GVM_MODE_BATCH) batch_open_ = true;
  return true;
}

int Manager::shutdown() {
  if (!started_) return GVM_OK;
  stop_.store(true, std::memory_order_release);
  ctl_->bell.fetch_add(1);
  futex_wake_all(&ctl_->bell);
  thread_.join();
  started_ = false;
  for (uint32_t r = 0; r < cfg_.nranks; ++r) {
    for (Job* j : ranks_[r].running) delete j;  // not reached: the service loop drained
    ranks_[r].running.clear();
  }
  dev_.reset();
  data_.clear();
  ctl_ = nullptr;
  ctl_seg_.close();
  return GVM_OK;
}

namespace {
double pct(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t rank = static_cast<size_t>(std::ceil(p / 100.0 * v.size()));
  if (rank < 1) rank = 1;
  return v[rank - 1];
}
}  // namespace

int Manager::stats_json(std::string* out) {
  if (!started_) return fail(GVM_ESTATE, "no manager runs in this process");
  if (std::this_thread::get_id() != thread_.get_id()) {
    // let the service thread retire finished batches first, so that the
    // counters cover every request answered so far
    std::unique_lock<std::mutex> fl(flush_mu_);
    const uint64_t gen = flush_done_;
    flush_req_.store(true, std::memory_order_release);
    ctl_->bell.fetch_add(1, std::memory_order_seq_cst);
    futex_wake_all(&ctl_->bell);
    // bounded by the wall clock: a wait on the system clock is a plain timed
    // condition wait, which thread checkers follow (a steady-clock wait is
    // not followed by some of them and reads as a lock held across it)
    flush_cv_.wait_until(fl, std::chrono::system_clock::now() + std::chrono::milliseconds(200),
                       [&] { return flush_done_ != gen || stop_.load(std::memory_order_acquire); });
  }
  std::lock_guard<std::mutex> lk(stats_mu_);
  char buf[512];
  std::string s = "{";
  s += "\"namespace\":\"" + ns_ + "\",\"device\":" + dev_->describe() + ",\"timing\":" + timing_json_;
  snprintf(buf, sizeof(buf), ",\"requests_done\":%llu,\"requests_failed\":%llu,\"batches\":%llu,\"peak_device_bytes\":%llu,\"arena_bytes\":%llu",
           (unsigned long long)n_done_, (unsigned long long)n_err_, (unsigned long long)n_batches_,
           (unsigned long long)std::max(peak_bytes_, arena_.peak()), (unsigned long long)arena_.total());
  s += buf;
  s += ",\"kernels\":{";
  bool first = true;
  for (int k = 0; k < kNumKernelIds; ++k) {
    const KernelStats& ks = kstats_[k];
    if (k == 0 && ks.launches == 0) continue;
    std::vector<double> all = lat_us_[k];
    snprintf(buf, sizeof(buf),
             "%s\"%s\":{\"launches\":%llu,\"requests\":%llu,\"device_ms\":%.6f,\"work_flop\":%.6e,\"work_bytes\":%.6e,"
             "\"latency_us\":{\"count\":%zu,\"p50\":%.3f,\"p99\":%.3f,\"max\":%.3f}}",
             first ? "" : ",", k == 0 ? "mixed_graph" : kernel_name(k), (unsigned long long)ks.launches, (unsigned long long)ks.requests,
             ks.device_ms, ks.work_flop, ks.work_bytes, all.size(), pct(all, 50), pct(all, 99), pct(all, 100));
    s += buf;
    first = false;
  }
  s += "}";
  snprintf(buf, sizeof(buf), ",\"admit_wait_us\":{\"count\":%zu,\"p50\":%.3f,\"p99\":%.3f,\"max\":%.3f}", wait_us_.size(),
           pct(wait_us_, 50), pct(wait_us_, 99), pct(wait_us_, 100));
  s += buf;
  // submit -> drained from the ring; last request of a batch drained -> batch admitted
  snprintf(buf, sizeof(buf), ",\"ring_us\":{\"count\":%zu,\"p50\":%.3f,\"p99\":%.3f},\"batch_admit_lag_us\":{\"count\":%zu,\"p50\":%.3f,\"p99\":%.3f}",
           ring_us_.size(), pct(ring_us_, 50), pct(ring_us_, 99), batch_lag_us_.size(), pct(batch_lag_us_, 50),
           pct(batch_lag_us_, 99));
  s += buf;
  // service iterations that retired or launched work: whole, and their completion part
  snprintf(buf, sizeof(buf), ",\"busy_iteration_us\":{\"count\":%zu,\"p50\":%.3f,\"p99\":%.3f,\"max\":%.3f,\"completion_p50\":%.3f,\"completion_p99\":%.3f}",
           iter_us_.size(), pct(iter_us_, 50), pct(iter_us_, 99), pct(iter_us_, 100), pct(iter_done_us_, 50),
           pct(iter_done_us_, 99));
  s += buf;
  // host side since the last reset: staging copies and the service thread's CPU time
  const CopyEngine::Stats cs = copy_.stats();
  const double wall = (now_ns() - stats_t0_ns_) * 1e-9;
  snprintf(buf, sizeof(buf),
           ",\"host\":{\"wall_s\":%.4f,\"copy_threads\":%d,\"copy_bytes\":%llu,\"copy_busy_s\":%.4f,\"copy_max_queue\":%zu,"
           "\"service_cpu_s\":%.4f}}",
           wall, copy_.threads(), (unsigned long long)cs.bytes, cs.busy_ns * 1e-9, cs.max_queue, (service_cpu_ns() - stats_cpu0_ns_) * 1e-9);
  s += buf;
  *out = s;
  return GVM_OK;
}

uint64_t Manager::service_cpu_ns() const {
  clockid_t cid;
  timespec ts{};
  if (!started_ || pthread_getcpuclockid(const_cast<std::thread&>(thread_).native_handle(), &cid) != 0 ||
      clock_gettime(cid, &ts) != 0)
    return 0;
  return static_cast<uint64_t>(ts.tv_sec) * 1000000000ull + static_cast<uint64_t>(ts.tv_nsec);
}

void Manager::reset_stats() {
  std::lock_guard<std::mutex> lk(stats_mu_);
  n_done_ = n_err_ = n_batches_ = 0;
  for (auto& v : lat_us_) v.clear();
  wait_us_.clear();
  ring_us_.clear();
  batch_lag_us_.clear();
  iter_us_.clear();
  iter_done_us_.clear();
  for (auto& k : kstats_) k = KernelStats{};
  peak_bytes_ = 0;
  trace_.clear();
  trace_next_ = 0;
  n_traced_ = 0;
  timing_json_ = "{}";
  copy_.reset_stats();
  stats_t0_ns_ = now_ns();
  stats_cpu0_ns_ = service_cpu_ns();
  // the device counters are reset on the service thread's next completion
  reset_pending_.store(true);
}

// Chrome trace-event JSON (read by Perfetto and chrome://tracing): process 1
// is the manager, one thread track per rank; each request is four complete
// ("X") slices on its rank's track, times in microseconds from the earliest
// submit in the file:
//   queued    submit -> admitted (ring, barrier or admission wait)
//   copy-in   admitted -> device work enqueued (shared memory -> pinned)
//   device    enqueued -> device work seen complete (H2D, kernel, D2H)
//   copy-out  device done -> result posted (pinned -> shared memory)
// A stage whose timestamps are missing (a rejected request) is left out.
int Manager::trace_dump(const char* path) {
  if (!started_) return fail(GVM_ESTATE, "no manager runs in this process");
  if (!path || !*path) return fail(GVM_EINVAL, "trace path is empty");
  std::vector<TraceRec> recs;
  uint64_t total = 0;
  {
    std::lock_guard<std::mutex> lk(stats_mu_);
    recs.reserve(trace_.size());
    for (size_t i = 0; i < trace_.size(); ++i) recs.push_back(trace_[(trace_next_ + i) % trace_.size()]);
    total = n_traced_;
  }
  FILE* f = fopen(path, "w");
  if (!f) return fail(GVM_ESYS, "cannot open %s for writing", path);
  uint64_t t0 = UINT64_MAX;
  for (const TraceRec& t : recs)
    if (t.t_submit && t.t_submit < t0) t0 = t.t_submit;
  if (t0 == UINT64_MAX) t0 = 0;
  fprintf(f, "{\"displayTimeUnit\":\"ns\",\"otherData\":{\"requests_traced\":%llu,\"requests_in_file\":%zu},"
             "\"traceEvents\":[\n", (unsigned long long)total, recs.size());
  fprintf(f, "{\"ph\":\"M\",\"pid\":1,\"name\":\"process_name\",\"args\":{\"name\":\"gvm manager %s\"}}", ns_.c_str());
  std::vector<int> named(cfg_.nranks, 0);
  for (const TraceRec& t : recs) {
    if (t.rank >= 0 && t.rank < static_cast<int>(cfg_.nranks) && !named[static_cast<size_t>(t.rank)]) {
      named[static_cast<size_t>(t.rank)] = 1;
      fprintf(f, ",\n{\"ph\":\"M\",\"pid\":1,\"tid\":%d,\"name\":\"thread_name\",\"args\":{\"name\":\"rank %d\"}}",
              t.rank, t.rank);
    }
    const uint64_t st[5] = {t.t_submit, t.t_admit, t.t_launch, t.t_device, t.t_done};
    static const char* const names[4] = {"queued", "copy-in", "device", "copy-out"};
    for (int k = 0; k < 4; ++k) {
      if (!st[k] || !st[k + 1] || st[k + 1] < st[k]) continue;
      fprintf(f,
              ",\n{\"ph\":\"X\",\"pid\":1,\"tid\":%d,\"name\":\"%s\",\"cat\":\"%s\",\"ts\":%.3f,\"dur\":%.3f,"
              "\"args\":{\"ticket\":%llu,\"n\":%llu,\"status\":%d}}",
              t.rank, names[k], t.kernel_id >= 1 && t.kernel_id <= 5 ? kernel_name(static_cast<int>(t.kernel_id)) : "?",
              (st[k] - t0) * 1e-3, (st[k + 1] - st[k]) * 1e-3, (unsigned long long)t.ticket, (unsigned long long)t.n,
              t.status);
    }
  }
  fprintf(f, "\n]}\n");
  const bool ok = !ferror(f);
  fclose(f);
  return ok ? GVM_OK : fail(GVM_ESYS, "write to %s failed", path);
}

}  // namespace gvm
