// HIP device of the manager: the single context of device 0, per-rank
// kernel streams, two compute streams for grouped launches, one copy stream
// per direction (FIFO, in the role of the copy engines of the execution
// model), one device arena, per-rank pinned staging, and the three enqueue
// policies (PS-1, PS-2 of Section 4.2.1, and the grouped persistent launch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "batch_plan.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace gvm {

namespace {

static_assert(kPlanMaxGroup == kMaxGroup, "the batch plan splits groups at the kernel-argument capacity");

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(GVM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct TimedLaunch {
  int kernel_id;
  hipEvent_t e0, e1;
  uint32_t requests;
  double flop, bytes;
};

struct EventState {
  uint64_t round;
  bool done;
  hipError_t err;
};

struct TimedCopy {
  int dir;  // 0 host->device, 1 device->host
  hipEvent_t e0, e1;
  uint64_t bytes;
  bool first;  // first piece of a request's copy (copies are counted per request)
};

struct Batch {
  std::map<hipEvent_t, EventState> state;  // polled completion events
  hipEvent_t span0 = nullptr, span1 = nullptr;  // device phase of the batch (batch_timing)
  std::vector<TimedCopy> copies;                // timed copies (batch_timing)
  std::vector<Job*> jobs;
  std::vector<hipEvent_t> done;   // per job (several jobs may share one event)
  std::vector<hipEvent_t> sync;   // events owned by the batch, recycled at the end
  std::vector<TimedLaunch> timed;
  std::vector<std::vector<hipEvent_t>> out_ev;  // per job: one event after each output piece
  std::vector<uint32_t> out_done;               // per job: leading output pieces seen complete
  size_t remaining = 0;
};

// Tile configuration of one grouped SGEMM launch, its requests sorted by
// size from the largest down (every configuration gives the same bits, so
// the choice is about speed alone).
//  * One size: the table's configuration of that size.
//  * Mixed sizes: 64x128x16 tiles with row-major B, a two-deep fetch and
//    registers held to four waves per SIMD (configuration 29), the smallest
//    tiles that still run near full rate.  The same tile at three waves per
//    SIMD (17) ran the 32-rank uneven launch 3.5 % slower (671-674 against
//    647-650 us), its pipelined sibling (25) slower again.  Small tiles
//    balance the short and the long tiles of a mix over the CUs, where
//    128x128 or larger tiles leave CUs idle at the end.
// Tuning override for mixed sizes: GVM_SGEMM_MIX_CONFIG=<index>.
constexpr int kMixConfig = 29;

int gemm_group_config(const std::vector<Job*>& v) {
  if (v.front()->req.n == v.back()->req.n) return gemm_config_for(v.front()->req.n);
  static const int env = [] {
    const char* e = getenv("GVM_SGEMM_MIX_CONFIG");
    return e ? atoi(e) : -1;
  }();
  return env >= 0 && env < gemm_config_count() ? env : kMixConfig;
}

// Grid cap of an SGEMM launch over mixed sizes: one workgroup per tile, so
// that the dispatcher hands the next tile to whichever CU frees up first
// (tiles of different sizes differ in k-length by up to 5x; a persistent
// grid deals them out statically).  GVM_SGEMM_MIX_GRID overrides.
int gemm_mix_grid() {
  static const int env = [] {
    const char* e = getenv("GVM_SGEMM_MIX_GRID");
    return e ? atoi(e) : 0;
  }();
  return env > 0 ? env : (1 << 24);
}

// Order of a grouped batch's launches: 0 = dealt over both compute streams,
// longest first (default); 1 = one stream, longest first; 2 = one stream,
// shortest first.  GVM_PLAN_SERIAL overrides.
int plan_serial() {
  static const int env = [] {
    const char* e = getenv("GVM_PLAN_SERIAL");
    return e ? atoi(e) : 0;
  }();
  return env;
}

class HipDevice final : public Device {
 public:
  ~HipDevice() override { close(); }

  int open(const gvm_config& cfg) override {
    cfg_ = cfg;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
      return fail(GVM_EDEVICE, "no HIP device visible (the HIP backend has no CPU fallback)");
    HIPCHK(hipSetDevice(0));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, 0));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(GVM_EDEVICE, "device 0 is %s; this library is built for gfx950 only", prop.gcnArchName);
    arch_ = prop.gcnArchName;
    cus_ = prop.multiProcessorCount;
    const int ns = cfg.nstreams ? static_cast<int>(cfg.nstreams) : std::min<int>(cfg.nranks, 8);
    for (int i = 0; i < ns; ++i) {
      hipStream_t s;
      HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      rank_streams_.push_back(s);
    }
    for (int i = 0; i < 2; ++i) {
      hipStream_t s;
      HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      compute_streams_.push_back(s);
    }
    HIPCHK(hipStreamCreateWithFlags(&h2d_, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&d2h_, hipStreamNonBlocking));
    if (cfg.latency_cus) {
      if (cus_ != kPartitionCus)
        return fail(GVM_EINVAL, "latency_cus needs a device of %d CUs (this one has %d)", kPartitionCus, cus_);
      if (cu_partition_masks(cfg.latency_cus, part_mask_[0], part_mask_[1]) != GVM_OK)
        return fail(GVM_EINVAL, "latency_cus %u is not a multiple of 32 below %d", cfg.latency_cus, kPartitionCus);
      // GVM_PARTITION_MASKS=0 keeps the two class streams but without CU
      // masks (for measuring what the masks add to the separate streams)
      const char* env = getenv("GVM_PARTITION_MASKS");
      part_masked_ = !(env && env[0] == '0');
      for (int p = 0; p < 2; ++p) {
        hipStream_t s;
        if (part_masked_) HIPCHK(hipExtStreamCreateWithCUMask(&s, kPartitionCus / 32, part_mask_[p]));
        else HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        part_streams_.push_back(s);
      }
    }
    HIPCHK(hipMalloc(reinterpret_cast<void**>(&arena_), cfg.hbm_budget_bytes));
    staging_.assign(cfg.nranks, nullptr);
    staging_bytes_ = cfg.staging_bytes ? cfg.staging_bytes : cfg.shm_bytes_per_rank;
    staging_bytes_ = align_up(staging_bytes_ + 2 * kAlign, 4096);
    int rc = prepare_kernels();
    if (rc != GVM_OK) return rc;
    return prepare_staging();
  }

  // Allocate every rank's pinned staging now and run one device-to-host copy
  // into all of it: the first DMA into freshly pinned pages runs at about a
  // third of the link rate, later ones at the full rate (57 GB/s).
  int prepare_staging() {
    hipStream_t s = compute_streams_[0];
    const uint64_t chunk = std::min<uint64_t>(cfg_.hbm_budget_bytes, 64ull << 20);
    for (int r = 0; r < static_cast<int>(staging_.size()); ++r) {
      uint8_t* p = staging(r);
      if (!p) return GVM_EDEVICE;
      for (uint64_t off = 0; off < staging_bytes_; off += chunk)
        HIPCHK(hipMemcpyAsync(p + off, arena_, std::min(chunk, staging_bytes_ - off), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return GVM_OK;
  }

  uint8_t* arena() override { return arena_; }

  // Pinned staging of a rank, allocated on first use.  Non-coherent
  // (coarse-grained) host memory: the device's copy engines move it to and
  // from HBM at the link's rate in both directions (57 GB/s device to host,
  // against 30 GB/s for coherent memory, 97 GB/s both ways at once), and the
  // staging is only ever touched by hipMemcpyAsync on the device side, whose
  // completion the host observes through events with the default system-scope
  // fence before it reads a result.  GVM_STAGING_COHERENT=1 takes coherent
  // memory instead (measurement).
  uint8_t* staging(int rank) override {
    if (rank < 0 || rank >= static_cast<int>(staging_.size())) return nullptr;
    if (!staging_[rank]) {
      static const unsigned flags = [] {
        const char* e = getenv("GVM_STAGING_COHERENT");
        return (e && e[0] == '1') ? hipHostMallocDefault : hipHostMallocNonCoherent;
      }();
      void* p = nullptr;
      if (hipHostMalloc(&p, staging_bytes_, flags) != hipSuccess) {
        fail(GVM_EDEVICE, "hipHostMalloc(%llu) failed", (unsigned long long)staging_bytes_);
        return nullptr;
      }
      staging_[rank] = static_cast<uint8_t*>(p);
    }
    return staging_[rank];
  }

  int stream_in(Job* j, uint64_t off, uint64_t bytes) override {
    // timing records wait in pre_copies_ until the job's batch exists
    const int rc = timed_copy(j->slot + off, j->pin + off, bytes, hipMemcpyHostToDevice, h2d_,
                              cfg_.batch_timing ? &pre_copies_[j] : nullptr, off == 0);
    if (rc != GVM_OK || off + bytes < j->lay.in_bytes || capturing_) return rc;
    // the last piece: an event after it, so that the job's kernel waits for
    // its own input and not for what was queued on the FIFO after it (the
    // next batch's inputs, with early copy-in); the job's batch owns it
    hipEvent_t e = nullptr;
    if (!free_sync_.empty()) {
      e = free_sync_.back();
      free_sync_.pop_back();
    } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      return fail(GVM_EDEVICE, "hipEventCreate failed");
    }
    HIPCHK(hipEventRecord(e, h2d_));
    j->in_done = e;
    return GVM_OK;
  }

  int out_pieces_done(Job* j) override {
    auto* b = static_cast<Batch*>(j->batch);
    if (!b) return static_cast<int>(j->out_pieces);
    const size_t i = static_cast<size_t>(j->done_index);
    const auto& evs = b->out_ev[i];
    uint32_t& done = b->out_done[i];
    // the events were tracked: their state is what the last polling round
    // (begin_poll) saw, so no runtime call per job here
    while (done < evs.size()) {
      auto it = b->state.find(evs[done]);
      if (it == b->state.end() || (!it->second.done && it->second.err == hipErrorNotReady)) break;
      if (!it->second.done)
        return fail(GVM_EDEVICE, "device-to-host copy failed: %s", hipGetErrorString(it->second.err));
      ++done;
    }
    return static_cast<int>(done);
  }

  int launch(std::vector<Job*>& jobs, int policy) override {
    if (jobs.empty()) return GVM_OK;
    if (broken_) {
      // after a capture that left a stream capturing nothing more is enqueued;
      // the jobs fail here, without a batch
      const int rc = fail(GVM_EDEVICE, "the device takes no more work after a failed batch capture");
      for (Job* j : jobs) {
        j->status = rc;
        j->batch = nullptr;
        if (j->in_done) free_sync_.push_back(static_cast<hipEvent_t>(j->in_done));
        j->in_done = nullptr;
      }
      return rc;
    }
    if (policy != GVM_POLICY_PS1 && policy != GVM_POLICY_PS2)
      std::stable_sort(jobs.begin(), jobs.end(), [](const Job* x, const Job* y) { return x->rank < y->rank; });
    if (jobs[0]->part >= 0 && part_streams_.size() == 2) ++part_launches_[jobs[0]->part];
    auto* b = new Batch;
    b->jobs = jobs;
    b->done.assign(jobs.size(), nullptr);
    b->out_ev.resize(jobs.size());
    b->out_done.assign(jobs.size(), 0);
    b->remaining = jobs.size();
    for (size_t i = 0; i < jobs.size(); ++i) {
      jobs[i]->batch = b;
      jobs[i]->done_index = static_cast<int>(i);
      jobs[i]->t_launch_ns = now_ns();
      if (jobs[i]->in_done) b->sync.push_back(static_cast<hipEvent_t>(jobs[i]->in_done));  // recycled with b
      auto pre = pre_copies_.find(jobs[i]);
      if (pre != pre_copies_.end()) {
        b->copies.insert(b->copies.end(), pre->second.begin(), pre->second.end());
        pre_copies_.erase(pre);
      }
    }
    int rc = GVM_OK;
    // device phase of the batch: every stream it uses starts after span0 and
    // span1 follows them all (batch_timing; not combined with graph replay)
    std::vector<hipStream_t> span_streams;
    const bool span = cfg_.batch_timing && !cfg_.use_graphs;
    if (span) {
      // only the streams that carry work of this batch (each extra stream
      // costs a cross-queue wait at both ends of the span)
      hipStream_t c0 = compute_streams_[0];
      bool any_in = false, any_out = false;
      for (Job* j : jobs) {
        any_in |= j->copy_in && (!j->local || policy == GVM_POLICY_PS1);
        any_out |= j->copy_out && (!j->local || policy == GVM_POLICY_PS1);
      }
      if (any_in) span_streams.push_back(h2d_);
      if (any_out) span_streams.push_back(d2h_);
      if (policy == GVM_POLICY_PS1 || policy == GVM_POLICY_PS2) {
        for (Job* j : jobs) {
          hipStream_t s = kernel_stream(j);
          if (std::find(span_streams.begin(), span_streams.end(), s) == span_streams.end()) span_streams.push_back(s);
        }
      } else if (jobs[0]->part >= 0 && part_streams_.size() == 2) {
        span_streams.push_back(part_streams_[static_cast<size_t>(jobs[0]->part)]);
      } else if (grouped_launches(jobs) > 1) {
        span_streams.push_back(compute_streams_[1]);
      }
      b->span0 = timed_event();
      b->span1 = timed_event();
      if (!b->span0 || !b->span1) rc = fail(GVM_EDEVICE, "hipEventCreate failed");
      if (rc == GVM_OK && hipEventRecord(b->span0, c0) != hipSuccess) rc = fail(GVM_EDEVICE, "event record failed");
      for (hipStream_t s : span_streams)
        if (rc == GVM_OK && hipStreamWaitEvent(s, b->span0, 0) != hipSuccess) rc = fail(GVM_EDEVICE, "stream wait failed");
    }
    if (rc != GVM_OK) {
    } else if (policy == GVM_POLICY_PS2) {
      // Per rank: copy-in (host-to-device FIFO) -> kernel (rank stream) ->
      // copy-out (device-to-host FIFO).  The FIFOs play the paper's copy
      // engines: rank i+1's input streams in while rank i computes and
      // rank i-1's result streams out.
      for (size_t i = 0; i < jobs.size() && rc == GVM_OK; ++i) {
        Job* j = jobs[i];
        hipStream_t s = kernel_stream(j);
        std::vector<Job*> one{j};
        if (j->local) {  // small: the whole chain on the rank stream
          rc = enqueue_in(j, s);
          if (rc == GVM_OK) rc = enqueue_kernels(one, {s}, b);
          if (rc == GVM_OK) rc = enqueue_out(j, s);
          if (rc == GVM_OK) rc = record_done(b, i, s);
          continue;
        }
        if (j->copy_in) {
          rc = enqueue_in(j, h2d_);
          if (rc == GVM_OK && j->in_done) {
            HIPCHK(hipStreamWaitEvent(s, static_cast<hipEvent_t>(j->in_done), 0));
          } else if (rc == GVM_OK) {
            rc = after(s, h2d_, b);
          }
        }
        if (rc == GVM_OK) rc = enqueue_kernels(one, {s}, b);
        if (rc == GVM_OK && j->copy_out) {
          rc = after(d2h_, s, b);
          if (rc == GVM_OK) rc = enqueue_out(j, d2h_);
          if (rc == GVM_OK) rc = record_done(b, i, d2h_);
        } else if (rc == GVM_OK) {
          rc = record_done(b, i, s);
        }
      }
    } else if (policy == GVM_POLICY_PS1) {
      // Phases: every copy-in, then every kernel (concurrently, one per rank
      // stream), then every copy-out.
      std::vector<hipStream_t> ks;
      for (Job* j : jobs)
        if (std::find(ks.begin(), ks.end(), kernel_stream(j)) == ks.end()) ks.push_back(kernel_stream(j));
      bool any_in = false, any_out = false;
      for (size_t i = 0; i < jobs.size() && rc == GVM_OK; ++i) {
        any_in |= jobs[i]->copy_in;
        any_out |= jobs[i]->copy_out;
        rc = enqueue_in(jobs[i], h2d_);
      }
      if (any_in)
        for (size_t k = 0; k < ks.size() && rc == GVM_OK; ++k) rc = after(ks[k], h2d_, b);
      for (size_t i = 0; i < jobs.size() && rc == GVM_OK; ++i) {
        std::vector<Job*> one{jobs[i]};
        rc = enqueue_kernels(one, {kernel_stream(jobs[i])}, b);
      }
      if (any_out)
        for (size_t k = 0; k < ks.size() && rc == GVM_OK; ++k) rc = after(d2h_, ks[k], b);
      for (size_t i = 0; i < jobs.size() && rc == GVM_OK; ++i) {
        if (jobs[i]->copy_out) {
          rc = enqueue_out(jobs[i], d2h_);
          if (rc == GVM_OK) rc = record_done(b, i, d2h_);
        } else {
          rc = record_done(b, i, kernel_stream(jobs[i]));
        }
      }
    } else {
      rc = launch_grouped(b);
    }
    if (span && rc == GVM_OK) {
      hipStream_t c0 = compute_streams_[0];
      for (hipStream_t s : span_streams) {
        hipEvent_t ev = sync_event(b);
        if (!ev || hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(c0, ev, 0) != hipSuccess) {
          rc = fail(GVM_EDEVICE, "span join failed");
          break;
        }
      }
      if (rc == GVM_OK && hipEventRecord(b->span1, c0) != hipSuccess) rc = fail(GVM_EDEVICE, "event record failed");
      if (rc == GVM_OK) {  // the jobs complete with the span
        track(b, b->span1, c0);
        for (size_t i = 0; i < jobs.size(); ++i) b->done[i] = b->span1;
      }
    }
    batches_.push_back(b);
    if (rc != GVM_OK) {
      // Device state is unknown after a failed enqueue: wait for what was
      // queued (unless a stream was left capturing, where a synchronisation
      // is not allowed), then fail every job of the batch.
      if (!broken_) (void)hipDeviceSynchronize();
      for (Job* j : jobs) j->status = rc;
      for (size_t i = 0; i < jobs.size(); ++i) b->done[i] = nullptr;
    }
    return rc;
  }

  int query(Job* j) override {
    auto* b = static_cast<Batch*>(j->batch);
    if (j->status != GVM_OK) return 1;
    hipEvent_t ev = b->done[j->done_index];
    if (!ev) return 1;
    auto it = b->state.find(ev);
    if (it == b->state.end()) {  // not tracked (cannot happen): ask directly
      const hipError_t e = hipEventQuery(ev);
      it = b->state.insert_or_assign(ev, EventState{0, e == hipSuccess, e}).first;
    }
    if (it->second.done) {
      if (!j->t_device_ns) j->t_device_ns = now_ns();
      return 1;
    }
    if (it->second.err == hipErrorNotReady) return 0;
    j->status = fail(GVM_EDEVICE, "device work failed: %s", hipGetErrorString(it->second.err));
    return -1;
  }

  // One polling round: per stream, settle the pending events in order.
  void begin_poll() override {
    for (auto& kv : fifo_) {
      auto& q = kv.second;
      while (!q.empty()) {
        FifoEntry& e = q.front();
        const hipError_t r = hipEventQuery(e.ev);
        if (r == hipErrorNotReady) break;
        e.b->state[e.ev] = EventState{0, r == hipSuccess, r};
        q.pop_front();
      }
    }
  }

  void finish(Job* j) override {
    auto* b = static_cast<Batch*>(j->batch);
    j->batch = nullptr;
    if (b && --b->remaining == 0) retire_q_.push_back(b);
  }

  bool flush_retired() override {
    if (retire_q_.empty()) return false;
    for (Batch* b : retire_q_) retire(b);
    retire_q_.clear();
    return true;
  }

  void drain() override { (void)hipDeviceSynchronize(); }

  void close() override {
    if (closed_) return;
    closed_ = true;
    (void)hipDeviceSynchronize();
    for (Batch* b : batches_) {
      for (hipEvent_t e : b->sync) (void)hipEventDestroy(e);
      for (auto& t : b->timed) {
        (void)hipEventDestroy(t.e0);
        (void)hipEventDestroy(t.e1);
      }
      for (auto& c : b->copies) {
        (void)hipEventDestroy(c.e0);
        (void)hipEventDestroy(c.e1);
      }
      if (b->span0) (void)hipEventDestroy(b->span0);
      if (b->span1) (void)hipEventDestroy(b->span1);
      delete b;
    }
    batches_.clear();
    retire_q_.clear();
    for (auto& kv : graphs_) {
      (void)hipGraphExecDestroy(kv.second.exec);
      (void)hipGraphDestroy(kv.second.graph);
      for (hipEvent_t e : kv.second.events) (void)hipEventDestroy(e);
    }
    graphs_.clear();
    graphs_cached_.store(0);
    for (auto& kv : pre_copies_)
      for (auto& t : kv.second) {
        (void)hipEventDestroy(t.e0);
        (void)hipEventDestroy(t.e1);
      }
    pre_copies_.clear();
    for (hipEvent_t e : free_sync_) (void)hipEventDestroy(e);
    for (hipEvent_t e : free_timed_) (void)hipEventDestroy(e);
    for (hipEvent_t e : free_marks_) (void)hipEventDestroy(e);
    free_marks_.clear();
    free_sync_.clear();
    free_timed_.clear();
    for (hipStream_t s : rank_streams_) (void)hipStreamDestroy(s);
    for (hipStream_t s : compute_streams_) (void)hipStreamDestroy(s);
    for (hipStream_t s : part_streams_) (void)hipStreamDestroy(s);
    part_streams_.clear();
    if (h2d_) (void)hipStreamDestroy(h2d_);
    if (d2h_) (void)hipStreamDestroy(d2h_);
    h2d_ = d2h_ = nullptr;
    rank_streams_.clear();
    compute_streams_.clear();
    if (arena_) (void)hipFree(arena_);
    arena_ = nullptr;
    for (uint8_t* p : staging_)
      if (p) (void)hipHostFree(p);
    staging_.clear();
  }

  const KernelStats* kernel_stats() const override { return stats_; }
  void reset_stats() override {
    for (auto& s : stats_) s = KernelStats{};
    batch_us_.clear();
    launch_us_.clear();
    for (int d = 0; d < 2; ++d) copy_ms_[d] = copy_bytes_[d] = 0.0, copy_n_[d] = 0, copy_us_[d].clear();
  }

  // Batch device phases, copy and launch durations (us, the last 512 of
  // each; the copies one entry per copy or piece), and copy totals.
  std::string timing_json() const override {
    auto list = [](const std::vector<double>& v) {
      std::string s = "[";
      const size_t first = v.size() > 512 ? v.size() - 512 : 0;
      for (size_t i = first; i < v.size(); ++i) {
        if (i > first) s += ",";
        s += std::to_string(v[i]);
      }
      return s + "]";
    };
    std::string s = "{\"batch_device_us\":" + list(batch_us_) + ",\"h2d_us\":" + list(copy_us_[0]) +
                    ",\"d2h_us\":" + list(copy_us_[1]) + ",\"launch_us\":" + list(launch_us_);
    char buf[256];
    snprintf(buf, sizeof(buf), ",\"h2d\":{\"count\":%llu,\"ms\":%.6f,\"bytes\":%.0f},\"d2h\":{\"count\":%llu,\"ms\":%.6f,\"bytes\":%.0f}}",
             (unsigned long long)copy_n_[0], copy_ms_[0], copy_bytes_[0], (unsigned long long)copy_n_[1], copy_ms_[1],
             copy_bytes_[1]);
    return s + buf;
  }
  std::string describe() const override {
    return "{\"backend\":\"hip\",\"arch\":\"" + arch_ + "\",\"cus\":" + std::to_string(cus_) +
           ",\"rank_streams\":" + std::to_string(rank_streams_.size()) +
           ",\"compute_streams\":" + std::to_string(compute_streams_.size()) +
           ",\"latency_cus\":" + std::to_string(part_streams_.empty() ? 0 : cfg_.latency_cus) +
           ",\"partition_masked\":" + std::string(part_masked_ ? "true" : "false") +
           ",\"partition_launches\":[" + std::to_string(part_launches_[0].load()) + "," + std::to_string(part_launches_[1].load()) + "]" +
           ",\"graphs_cached\":" + std::to_string(graphs_cached_.load()) + ",\"graph_captures\":" + std::to_string(graph_captures_.load()) +
           ",\"graph_launches\":" + std::to_string(graph_launches_.load()) + "}";
  }

 private:
  hipStream_t rank_stream(int rank) { return rank_streams_[static_cast<size_t>(rank) % rank_streams_.size()]; }

  // The stream a job's kernel runs on under PS-1 / PS-2: its rank's stream,
  // or its CU partition's stream when the device is partitioned.
  hipStream_t kernel_stream(const Job* j) {
    if (j->part >= 0 && part_streams_.size() == 2) return part_streams_[static_cast<size_t>(j->part)];
    return rank_stream(j->rank);
  }

  // An untimed event for ordering streams, owned by batch `b` and recycled
  // when the batch retires.  During a stream capture the event is created
  // fresh and owned by the graph being built instead: it is never handed to
  // an eager batch while that graph exists.
  hipEvent_t sync_event(Batch* b) {
    hipEvent_t e = nullptr;
    if (capturing_) {
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        fail(GVM_EDEVICE, "hipEventCreate failed");
        return nullptr;
      }
      capture_events_.push_back(e);
      return e;
    }
    if (!free_sync_.empty()) {
      e = free_sync_.back();
      free_sync_.pop_back();
    } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      fail(GVM_EDEVICE, "hipEventCreate failed");
      return nullptr;
    }
    b->sync.push_back(e);
    return e;
  }

  hipEvent_t timed_event() {
    hipEvent_t e = nullptr;
    if (!free_timed_.empty()) {
      e = free_timed_.back();
      free_timed_.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      return nullptr;
    }
    return e;
  }

  // A timing mark around a kernel launch, read only by hipEventElapsedTime:
  // no system-scope fence when it is reached (a fence writes back and
  // invalidates the caches, which added 10-14 us to a launch's measured
  // time on some devices).  Nothing waits on it or queries it; the stream
  // order after a launch comes from ordinary events.
  hipEvent_t launch_mark() {
    hipEvent_t e = nullptr;
    if (!free_marks_.empty()) {
      e = free_marks_.back();
      free_marks_.pop_back();
    } else if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
      return nullptr;
    }
    return e;
  }

  // Number of grouped launches the grouped policy makes for `jobs`.
  static size_t grouped_launches(const std::vector<Job*>& jobs) {
    std::vector<PlanJob> pj;
    for (const Job* j : jobs) pj.push_back(plan_job(j));
    return plan_groups(pj, 2).size();
  }

  // `waiter` continues only after everything enqueued so far on `producer`.
  int after(hipStream_t waiter, hipStream_t producer, Batch* b) {
    hipEvent_t e = sync_event(b);
    if (!e) return GVM_EDEVICE;
    HIPCHK(hipEventRecord(e, producer));
    HIPCHK(hipStreamWaitEvent(waiter, e, 0));
    return GVM_OK;
  }

  int record_done(Batch* b, size_t i, hipStream_t s) {
    hipEvent_t e = sync_event(b);
    if (!e) return GVM_EDEVICE;
    HIPCHK(hipEventRecord(e, s));
    b->done[i] = e;
    track(b, e, s);
    return GVM_OK;
  }

  // Completion events in the order they were recorded on each stream; an
  // event can only complete after every earlier one of its stream, so a
  // polling round asks the runtime about the oldest pending one per stream.
  void track(Batch* b, hipEvent_t ev, hipStream_t s) {
    if (b->state.count(ev)) return;
    b->state[ev] = EventState{0, false, hipErrorNotReady};
    fifo_[s].push_back(FifoEntry{b, ev});
  }

  // One copy of a job between its pinned staging and its device slot; with
  // batch_timing (and outside a capture) bracketed by timing events.
  // `into` receives the timing record (a batch's list, or the pre-launch
  // list of a piecewise input); `first` marks a request's first piece.
  int timed_copy(void* dst, const void* src, uint64_t bytes, hipMemcpyKind kind, hipStream_t s,
                 std::vector<TimedCopy>* into, bool first = true) {
    TimedCopy t{kind == hipMemcpyHostToDevice ? 0 : 1, nullptr, nullptr, bytes, first};
    const bool timed = cfg_.batch_timing && !capturing_ && into;
    if (timed) {
      t.e0 = timed_event();
      t.e1 = timed_event();
      if (!t.e0 || !t.e1) return fail(GVM_EDEVICE, "hipEventCreate failed");
      HIPCHK(hipEventRecord(t.e0, s));
    }
    HIPCHK(hipMemcpyAsync(dst, src, bytes, kind, s));
    if (timed) {
      HIPCHK(hipEventRecord(t.e1, s));
      into->push_back(t);
    }
    return GVM_OK;
  }

  int enqueue_in(Job* j, hipStream_t s) {
    if (!j->copy_in || j->pieces) return GVM_OK;  // a piecewise input is queued as it lands
    return timed_copy(j->slot, j->pin, j->lay.in_bytes, hipMemcpyHostToDevice, s, &static_cast<Batch*>(j->batch)->copies);
  }

  int enqueue_out(Job* j, hipStream_t s) {
    if (!j->copy_out) return GVM_OK;
    const uint64_t o = slot_out_offset(j->lay);
    auto* b = static_cast<Batch*>(j->batch);
    if (!j->out_pieces)
      return timed_copy(j->pin + o, j->slot + o, j->lay.out_bytes, hipMemcpyDeviceToHost, s, &b->copies);
    // piecewise: an event after each piece lets the host copy of the
    // leading pieces start while the rest is still on the link
    auto& evs = b->out_ev[static_cast<size_t>(j->done_index)];
    for (uint32_t i = 0; i < j->out_pieces; ++i) {
      const uint64_t off = static_cast<uint64_t>(i) * piece_bytes();
      const int rc = timed_copy(j->pin + o + off, j->slot + o + off, std::min<uint64_t>(piece_bytes(), j->lay.out_bytes - off),
                                hipMemcpyDeviceToHost, s, &b->copies, i == 0);
      if (rc != GVM_OK) return rc;
      hipEvent_t e = sync_event(b);
      if (!e) return GVM_EDEVICE;
      HIPCHK(hipEventRecord(e, s));
      evs.push_back(e);
      if (!capturing_) track(b, e, s);  // settled by the per-stream polling rounds
    }
    return GVM_OK;
  }

  // The plan's view of a job.
  static PlanJob plan_job(const Job* j) {
    const int k = static_cast<int>(j->req.kernel_id);
    return PlanJob{k, j->req.n, j->copy_in, j->copy_out, j->local, j->pieces && j->copy_in, j->out_pieces > 0};
  }

  // One grouped launch per kernel id, at most kMaxGroup requests each, dealt
  // round robin to `streams` (PS-1 and PS-2 call it with one job and its own
  // stream).  Each launch is timed.
  int enqueue_kernels(const std::vector<Job*>& jobs, const std::vector<hipStream_t>& streams, Batch* b) {
    std::vector<PlanJob> pj;
    for (const Job* j : jobs) pj.push_back(plan_job(j));
    for (const PlanGroup& g : plan_groups(pj, static_cast<int>(streams.size()))) {
      const int rc = launch_group(g, jobs, streams[static_cast<size_t>(g.stream)], b, true);
      if (rc != GVM_OK) return rc;
    }
    return GVM_OK;
  }

  // One grouped launch of the requests `g.jobs` of `jobs` on stream `s`.
  // `timed`: bracketed by timing marks (a caller that orders other work
  // after the launch records an event of its own).
  int launch_group(const PlanGroup& g, const std::vector<Job*>& jobs, hipStream_t s, Batch* b, bool timed) {
    const int k = g.kernel_id;
    const size_t cnt = g.jobs.size();
    if (cnt == 0 || cnt > static_cast<size_t>(kMaxGroup)) return fail(GVM_EINVAL, "group of %zu requests", cnt);
    std::vector<Job*> v;
    for (int i : g.jobs) v.push_back(jobs[static_cast<size_t>(i)]);
    TimedLaunch t{};
    t.kernel_id = k;
    t.requests = static_cast<uint32_t>(cnt);
    if (timed) {
      t.e0 = launch_mark();
      t.e1 = launch_mark();
      if (!t.e0 || !t.e1) return fail(GVM_EDEVICE, "hipEventCreate failed");
    }
    for (Job* j : v) {
      double f, by;
      request_work(k, j->req.n, &f, &by);
      t.flop += f;
      t.bytes += by;
    }
    // The descriptors are built first, so that the opening mark is recorded
    // right before the launch call: host work between the two would be
    // counted as the kernel's time when the stream is idle.
    hipError_t e = hipSuccess;
    auto mark = [&]() -> hipError_t { return timed ? hipEventRecord(t.e0, s) : hipSuccess; };
    if (k == GVM_K_VECADD || k == GVM_K_VECMUL) {
      VecGroup vg{};
      vg.count = static_cast<uint32_t>(cnt);
      for (size_t i = 0; i < cnt; ++i) {
        float* in = reinterpret_cast<float*>(v[i]->slot);
        vg.d[i].a = in;
        vg.d[i].b = in + v[i]->req.n;
        vg.d[i].c = reinterpret_cast<float*>(v[i]->slot + slot_out_offset(v[i]->lay));
        vg.d[i].n = v[i]->req.n;
      }
      finalize_vec_group(vg);
      if ((e = mark()) == hipSuccess) e = (k == GVM_K_VECADD) ? launch_vecadd_group(vg, s) : launch_vecmul_group(vg, s);
    } else if (k == GVM_K_BLACKSCHOLES) {
      BsGroup bg{};
      bg.count = static_cast<uint32_t>(cnt);
      bg.rate = cfg_.bs_rate;
      bg.volatility = cfg_.bs_volatility;
      for (size_t i = 0; i < cnt; ++i) {
        const uint64_t n = v[i]->req.n;
        float* in = reinterpret_cast<float*>(v[i]->slot);
        float* out = reinterpret_cast<float*>(v[i]->slot + slot_out_offset(v[i]->lay));
        bg.d[i].S = in;
        bg.d[i].K = in + n;
        bg.d[i].T = in + 2 * n;
        bg.d[i].call = out;
        bg.d[i].put = out + n;
        bg.d[i].n = n;
      }
      finalize_bs_group(bg);
      if ((e = mark()) == hipSuccess) e = launch_bs_group(bg, s);
    } else if (k == GVM_K_SGEMM) {
      GemmGroup gg{};
      gg.count = static_cast<uint32_t>(cnt);
      for (size_t i = 0; i < cnt; ++i) {
        const uint64_t n = v[i]->req.n;
        float* in = reinterpret_cast<float*>(v[i]->slot);
        gg.d[i].A = in;
        gg.d[i].B = in + n * n;
        gg.d[i].C = reinterpret_cast<float*>(v[i]->slot + slot_out_offset(v[i]->lay));
        gg.d[i].n = static_cast<uint32_t>(n);
      }
      const int cfgi = gemm_group_config(v);
      finalize_gemm_group(gg, cfgi);
      const bool mixed = v.front()->req.n != v.back()->req.n;
      if ((e = mark()) == hipSuccess) e = launch_sgemm_group(gg, cfgi, s, mixed ? gemm_mix_grid() : 0);
    } else if (k == GVM_K_EP) {
      EpGroup eg{};
      eg.count = static_cast<uint32_t>(cnt);
      for (size_t i = 0; i < cnt; ++i) {
        eg.d[i].key = reinterpret_cast<const uint64_t*>(v[i]->slot);
        eg.d[i].out = reinterpret_cast<uint64_t*>(v[i]->slot + slot_out_offset(v[i]->lay));
        eg.d[i].partial = reinterpret_cast<uint64_t*>(v[i]->slot + slot_scratch_offset(v[i]->lay));
        eg.d[i].n = v[i]->req.n;
      }
      finalize_ep_group(eg);
      if ((e = mark()) == hipSuccess) e = launch_ep_group(eg, s);
    } else {
      return fail(GVM_EINVAL, "unknown kernel id %d", k);
    }
    if (e != hipSuccess) return fail(GVM_EDEVICE, "kernel launch (%s): %s", kernel_name(k), hipGetErrorString(e));
    if (timed) {
      HIPCHK(hipEventRecord(t.e1, s));
      b->timed.push_back(t);
    }
    return GVM_OK;
  }

  // Grouped policy: the batch plan (copy-ins, grouped launches on the two
  // compute streams, copy-outs, completions), executed eagerly, or with
  // use_graphs captured once per batch template (ranks, kernels, sizes,
  // copies, buffers) and replayed, with the piecewise copies around it.
  int launch_grouped(Batch* b) {
    std::vector<Job*>& jobs = b->jobs;
    std::vector<PlanJob> pj;
    for (const Job* j : jobs) pj.push_back(plan_job(j));
    hipStream_t st[kPlanStreams] = {compute_streams_[0], compute_streams_[1], h2d_, d2h_};
    if (jobs[0]->part >= 0 && part_streams_.size() == 2)
      st[kPlanC0] = st[kPlanC1] = part_streams_[static_cast<size_t>(jobs[0]->part)];
    if (!cfg_.use_graphs) {
      const int ser = plan_serial();
      const BatchPlan p = plan_grouped(pj, false, ser ? 1 : 2, ser != 2);
      PlanEvents ev(p);
      return run_ops(p.ops, p, st, b, true, ev);
    }

    hipStream_t c0 = compute_streams_[0];
    const BatchPlan p = plan_grouped(pj, true);
    PlanEvents ev(p);
    int rc = run_ops(p.pre, p, st, b, false, ev);
    if (rc != GVM_OK) return rc;
    std::string key = graph_key(jobs);
    auto it = graphs_.find(key);
    if (it == graphs_.end()) {
      if (graphs_.size() >= kMaxGraphs) evict_graph();
      HIPCHK(hipStreamBeginCapture(c0, hipStreamCaptureModeThreadLocal));
      capturing_ = true;
      capture_events_.clear();
      rc = run_ops(p.ops, p, st, b, false, ev);
      capturing_ = false;
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(c0, &g);
      std::vector<hipEvent_t> evs;
      evs.swap(capture_events_);
      // Whatever went wrong, no stream of the batch may stay in capture mode:
      // work enqueued later on such a stream would be added to a graph that
      // no longer exists.  If one does, the device stops taking work.
      for (hipStream_t s : {compute_streams_[0], compute_streams_[1], h2d_, d2h_}) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) broken_ = true;
      }
      if (broken_) {
        if (g) (void)hipGraphDestroy(g);
        return fail(GVM_EDEVICE, "a stream was left capturing after the batch capture; the device takes no more work");
      }
      if (rc != GVM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        for (hipEvent_t x : evs) (void)hipEventDestroy(x);
        return rc != GVM_OK ? rc : fail(GVM_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
      }
      hipGraphExec_t ex = nullptr;
      const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        for (hipEvent_t x : evs) (void)hipEventDestroy(x);
        return fail(GVM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
      }
      it = graphs_.emplace(key, GraphEntry{g, ex, 0, std::move(evs)}).first;
      graphs_cached_.store(graphs_.size());
      ++graph_captures_;
    }
    it->second.last_use = ++graph_clock_;
    TimedLaunch t{};
    t.kernel_id = static_cast<int>(jobs[0]->req.kernel_id);
    for (Job* j : jobs) {
      if (static_cast<int>(j->req.kernel_id) != t.kernel_id) t.kernel_id = 0;  // mixed batch
      double f, by;
      request_work(static_cast<int>(j->req.kernel_id), j->req.n, &f, &by);
      t.flop += f;
      t.bytes += by;
    }
    t.requests = static_cast<uint32_t>(jobs.size());
    t.e0 = launch_mark();
    t.e1 = launch_mark();
    if (!t.e0 || !t.e1) return fail(GVM_EDEVICE, "hipEventCreate failed");
    HIPCHK(hipEventRecord(t.e0, c0));
    HIPCHK(hipGraphLaunch(it->second.exec, c0));
    HIPCHK(hipEventRecord(t.e1, c0));
    b->timed.push_back(t);
    ++graph_launches_;
    return run_ops(p.post, p, st, b, false, ev);
  }

  // Device events of a plan's event ids, and the stream each was recorded on.
  struct PlanEvents {
    explicit PlanEvents(const BatchPlan& p)
        : ev(static_cast<size_t>(p.events), nullptr), stream(static_cast<size_t>(p.events), nullptr) {}
    std::vector<hipEvent_t> ev;
    std::vector<hipStream_t> stream;
  };

  // Execute plan operations on the streams `st` (indexed by PlanStream).
  // `timed`: launches are bracketed by timing events (eager batches only).
  int run_ops(const std::vector<PlanOp>& ops, const BatchPlan& p, const hipStream_t* st, Batch* b, bool timed,
              PlanEvents& pe) {
    std::vector<Job*>& jobs = b->jobs;
    for (const PlanOp& o : ops) {
      hipStream_t s = st[o.stream];
      int rc = GVM_OK;
      switch (o.kind) {
        case kOpRecord: {
          hipEvent_t e = sync_event(b);
          if (!e) return GVM_EDEVICE;
          HIPCHK(hipEventRecord(e, s));
          pe.ev[static_cast<size_t>(o.ev)] = e;
          pe.stream[static_cast<size_t>(o.ev)] = s;
          break;
        }
        case kOpWait:
          HIPCHK(hipStreamWaitEvent(s, pe.ev[static_cast<size_t>(o.ev)], 0));
          break;
        case kOpCopyIn:
          rc = enqueue_in(jobs[static_cast<size_t>(o.job)], s);
          break;
        case kOpCopyOut:
          rc = enqueue_out(jobs[static_cast<size_t>(o.job)], s);
          break;
        case kOpLaunch: {
          rc = launch_group(p.groups[static_cast<size_t>(o.group)], jobs, s, b, timed);
          if (rc == GVM_OK && o.ev >= 0) {  // the end of the launch on its stream
            hipEvent_t end = sync_event(b);
            if (!end) return GVM_EDEVICE;
            HIPCHK(hipEventRecord(end, s));
            pe.ev[static_cast<size_t>(o.ev)] = end;
            pe.stream[static_cast<size_t>(o.ev)] = s;
          }
          break;
        }
        case kOpDone:
          if (o.ev >= 0) {
            b->done[static_cast<size_t>(o.job)] = pe.ev[static_cast<size_t>(o.ev)];
            track(b, pe.ev[static_cast<size_t>(o.ev)], pe.stream[static_cast<size_t>(o.ev)]);
          } else {
            rc = record_done(b, static_cast<size_t>(o.job), s);
          }
          break;
        default:
          return fail(GVM_EINVAL, "unknown plan operation %d", o.kind);
      }
      if (rc != GVM_OK) return rc;
    }
    return GVM_OK;
  }

  static std::string graph_key(const std::vector<Job*>& jobs) {
    std::string key;
    for (const Job* j : jobs) {
      const uint64_t f[7] = {static_cast<uint64_t>(j->rank), j->req.kernel_id, j->req.n,
                             static_cast<uint64_t>(j->copy_in) | (static_cast<uint64_t>(j->copy_out) << 1),
                             reinterpret_cast<uint64_t>(j->slot), reinterpret_cast<uint64_t>(j->pin),
                             static_cast<uint64_t>(gemm_config_for(j->req.n))};
      key.append(reinterpret_cast<const char*>(f), sizeof(f));
    }
    return key;
  }

  void evict_graph() {
    auto victim = graphs_.begin();
    for (auto it = graphs_.begin(); it != graphs_.end(); ++it)
      if (it->second.last_use < victim->second.last_use) victim = it;
    (void)hipStreamSynchronize(compute_streams_[0]);  // no launch of it may be pending
    (void)hipGraphExecDestroy(victim->second.exec);
    (void)hipGraphDestroy(victim->second.graph);
    for (hipEvent_t e : victim->second.events) (void)hipEventDestroy(e);
    graphs_.erase(victim);
    graphs_cached_.store(graphs_.size());
  }

  void retire(Batch* b) {
    for (auto& kv : fifo_) {
      auto& q = kv.second;
      for (auto it = q.begin(); it != q.end();) it = (it->b == b) ? q.erase(it) : std::next(it);
    }
    for (auto& t : b->timed) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, t.e0, t.e1) == hipSuccess && t.kernel_id >= 0 && t.kernel_id < kNumKernelIds) {
        // kernel id 0 collects graph launches of mixed batches
        KernelStats& ks = stats_[t.kernel_id];
        ks.launches += 1;
        ks.requests += t.requests;
        ks.device_ms += ms;
        ks.work_flop += t.flop;
        ks.work_bytes += t.bytes;
        if (launch_us_.size() < 65536) launch_us_.push_back(ms * 1e3);
      }
      free_marks_.push_back(t.e0);
      free_marks_.push_back(t.e1);
    }
    if (b->span0 && b->span1) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, b->span0, b->span1) == hipSuccess && batch_us_.size() < 65536)
        batch_us_.push_back(ms * 1e3);
      free_timed_.push_back(b->span0);
      free_timed_.push_back(b->span1);
    }
    for (auto& c : b->copies) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, c.e0, c.e1) == hipSuccess) {
        copy_ms_[c.dir] += ms;
        copy_bytes_[c.dir] += static_cast<double>(c.bytes);
        copy_n_[c.dir] += c.first ? 1 : 0;
        if (copy_us_[c.dir].size() < 65536) copy_us_[c.dir].push_back(ms * 1e3);
      }
      free_timed_.push_back(c.e0);
      free_timed_.push_back(c.e1);
    }
    for (hipEvent_t e : b->sync) free_sync_.push_back(e);
    batches_.erase(std::remove(batches_.begin(), batches_.end(), b), batches_.end());
    delete b;
  }

  // Load every kernel's code object now, as the manager of Section 5 prepares
  // the kernels at initialisation: one tiny launch of each on arena memory.
  int prepare_kernels() {
    if (cfg_.hbm_budget_bytes < (1u << 20)) return GVM_OK;
    hipStream_t s = compute_streams_[0];
    float* base = reinterpret_cast<float*>(arena_);
    HIPCHK(hipMemsetAsync(base, 0, 1 << 20, s));
    VecGroup vg{};
    vg.count = 1;
    vg.d[0] = VecDesc{base, base + 64, base + 128, 64, 0};
    finalize_vec_group(vg);
    HIPCHK(launch_vecadd_group(vg, s));
    HIPCHK(launch_vecmul_group(vg, s));
    BsGroup bg{};
    bg.count = 1;
    bg.rate = cfg_.bs_rate;
    bg.volatility = cfg_.bs_volatility;
    bg.d[0] = BsDesc{base, base + 64, base + 128, base + 192, base + 256, 64, 0};
    finalize_bs_group(bg);
    HIPCHK(launch_bs_group(bg, s));
    for (int c = 0; c < gemm_config_count(); ++c) {
      GemmGroup gg{};
      gg.count = 1;
      gg.d[0] = GemmDesc{base, base + 4096, base + 8192, 64, 0, 0, 0};
      finalize_gemm_group(gg, c);
      HIPCHK(launch_sgemm_group(gg, c, s));
    }
    EpGroup eg{};
    eg.count = 1;
    uint64_t* w = reinterpret_cast<uint64_t*>(arena_);
    eg.d[0] = EpDesc{w, w + 16, w + 64, 64, 0, 0};  // key words are zero (memset above)
    finalize_ep_group(eg);
    HIPCHK(launch_ep_group(eg, s));
    HIPCHK(hipStreamSynchronize(s));
    return GVM_OK;
  }

  gvm_config cfg_{};
  std::string arch_;
  int cus_ = 0;
  bool closed_ = false;
  std::vector<hipStream_t> rank_streams_;
  std::vector<hipStream_t> compute_streams_;
  std::vector<hipStream_t> part_streams_;      // CU-masked: [0] latency class, [1] the rest (latency_cus)
  uint32_t part_mask_[2][kPartitionCus / 32] = {};
  std::atomic<uint64_t> part_launches_[2] = {};  // counters read by describe() on the API thread
  bool part_masked_ = false;
  hipStream_t h2d_ = nullptr, d2h_ = nullptr;  // copy FIFOs, one per direction
  std::map<const Job*, std::vector<TimedCopy>> pre_copies_;  // timed input pieces of jobs not yet launched
  std::vector<Batch*> retire_q_;                              // finished batches not yet retired
  size_t next_cs_ = 0;
  struct FifoEntry {
    Batch* b;
    hipEvent_t ev;
  };
  std::map<hipStream_t, std::deque<FifoEntry>> fifo_;
  bool capturing_ = false;
  std::vector<hipEvent_t> capture_events_;  // events recorded during the capture in progress
  bool broken_ = false;                     // a stream was left capturing: no more device work
  std::vector<double> batch_us_, launch_us_, copy_us_[2];
  double copy_ms_[2] = {0, 0}, copy_bytes_[2] = {0, 0};
  uint64_t copy_n_[2] = {0, 0};
  uint8_t* arena_ = nullptr;
  std::vector<uint8_t*> staging_;
  uint64_t staging_bytes_ = 0;
  std::vector<hipEvent_t> free_sync_;
  std::vector<hipEvent_t> free_timed_;
  std::vector<hipEvent_t> free_marks_;  // launch_mark() events
  std::vector<Batch*> batches_;
  KernelStats stats_[kNumKernelIds];
  struct GraphEntry {
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t last_use;
    std::vector<hipEvent_t> events;  // recorded during its capture; destroyed with the graph
  };
  static constexpr size_t kMaxGraphs = 32;
  std::map<std::string, GraphEntry> graphs_;
  uint64_t graph_clock_ = 0;
  std::atomic<uint64_t> graph_captures_{0}, graph_launches_{0};
  std::atomic<size_t> graphs_cached_{0};  // graphs_.size(), for describe()
};

}  // namespace

std::unique_ptr<Device> make_hip_device() { return std::unique_ptr<Device>(new HipDevice()); }

}  // namespace gvm
