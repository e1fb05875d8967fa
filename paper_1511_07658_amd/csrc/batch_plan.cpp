#include "batch_plan.hpp"

#include <algorithm>
#include <map>

#include "gvm.h"

namespace gvm {

namespace {

// Rough device time of one request (us) at sustained rates (FP32 MFMA 110
// TFLOP/s, HBM 5 TB/s, 120 G EP pairs/s), only to order the launches.
double job_us(const PlanJob& j) {
  const double n = static_cast<double>(j.n);
  switch (j.kernel_id) {
    case GVM_K_SGEMM: return 2.0 * n * n * n / 110e6;
    case GVM_K_BLACKSCHOLES: return 20.0 * n / 5e6;
    case GVM_K_EP: return n / 120e3;
    default: return 12.0 * n / 5e6;
  }
}

}  // namespace

std::vector<PlanGroup> plan_groups(const std::vector<PlanJob>& jobs, int nstreams, bool longest_first) {
  // One grouped launch per kernel id (an SGEMM request gets the same bits
  // from every tile configuration, so any sizes may share one launch).
  std::map<int, std::vector<int>> classes;
  for (size_t i = 0; i < jobs.size(); ++i) classes[jobs[i].kernel_id].push_back(static_cast<int>(i));
  std::vector<PlanGroup> out;
  for (auto& kv : classes) {
    std::vector<int>& v = kv.second;
    if (kv.first == GVM_K_SGEMM) {  // largest first, so the longest tiles start first
      std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return jobs[x].n > jobs[y].n; });
    }
    for (size_t base = 0; base < v.size(); base += kPlanMaxGroup) {
      PlanGroup g;
      g.kernel_id = kv.first;
      const size_t end = std::min(v.size(), base + kPlanMaxGroup);
      g.jobs.assign(v.begin() + static_cast<long>(base), v.begin() + static_cast<long>(end));
      out.push_back(std::move(g));
    }
  }
  // the longest launch is enqueued first (its workgroups are dispatched
  // before a concurrent short launch floods the CUs), then dealt round robin
  std::vector<double> us(out.size(), 0.0);
  for (size_t g = 0; g < out.size(); ++g)
    for (int j : out[g].jobs) us[g] += job_us(jobs[static_cast<size_t>(j)]);
  std::vector<size_t> order(out.size());
  for (size_t g = 0; g < order.size(); ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t b) { return longest_first ? us[a] > us[b] : us[a] < us[b]; });
  std::vector<PlanGroup> sorted;
  for (size_t k = 0; k < order.size(); ++k) {
    sorted.push_back(std::move(out[order[k]]));
    sorted.back().stream = static_cast<int>(k) % std::max(nstreams, 1);
  }
  return sorted;
}

BatchPlan plan_grouped(const std::vector<PlanJob>& jobs, bool graph, int compute_streams, bool longest_first) {
  BatchPlan p;
  p.groups = plan_groups(jobs, compute_streams == 1 ? 1 : 2, longest_first);
  p.stream_of.assign(jobs.size(), kPlanC0);
  for (const PlanGroup& g : p.groups)
    for (int j : g.jobs) p.stream_of[static_cast<size_t>(j)] = g.stream == 0 ? kPlanC0 : kPlanC1;

  std::vector<PlanOp>* list = &p.ops;
  auto op = [&](int kind, int stream, int ev = -1, int job = -1, int group = -1) {
    list->push_back(PlanOp{kind, stream, ev, job, group});
  };
  auto record = [&](int stream) {
    const int e = p.events++;
    op(kOpRecord, stream, e);
    return e;
  };

  bool any_pieces = false;
  for (const PlanJob& j : jobs) any_pieces |= j.copy_in && j.pieces;
  if (graph) {
    if (any_pieces) {  // eager, before the launch: the graph starts after the input pieces
      list = &p.pre;
      op(kOpWait, kPlanC0, record(kPlanH2D));
      list = &p.ops;
    }
    const int fork = record(kPlanC0);  // the other streams join the capture through C0
    for (int s : {kPlanH2D, kPlanD2H, kPlanC1}) op(kOpWait, s, fork);
  }

  // copy-ins in job order: small ones on C0 ahead of its kernels, the rest on
  // the H2D FIFO (a piecewise input is already queued there)
  bool fifo_in = false, local_in = false;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const PlanJob& j = jobs[i];
    if (!j.copy_in) continue;
    if (j.local) {
      local_in = true;
      op(kOpCopyIn, kPlanC0, -1, static_cast<int>(i));
    } else if (!j.pieces) {
      fifo_in = true;
      op(kOpCopyIn, kPlanH2D, -1, static_cast<int>(i));
    } else if (!graph) {
      fifo_in = true;  // the wait below covers the pieces queued earlier
    }
  }
  if (local_in && p.groups.size() > 1) op(kOpWait, kPlanC1, record(kPlanC0));  // C1's kernels may read C0's copies
  if (fifo_in) {
    const int e = record(kPlanH2D);
    op(kOpWait, kPlanC0, e);
    op(kOpWait, kPlanC1, e);
  }

  // grouped launches; the last one on each compute stream marks the end of
  // that stream's kernels
  int last[2] = {-1, -1};
  for (size_t g = 0; g < p.groups.size(); ++g) {
    const int s = p.groups[g].stream == 0 ? kPlanC0 : kPlanC1;
    op(kOpLaunch, s, -1, -1, static_cast<int>(g));
    last[s] = static_cast<int>(p.ops.size() - 1);
  }
  int kend[2] = {-1, -1};
  for (int c = 0; c < 2; ++c)
    if (last[c] >= 0) kend[c] = p.ops[static_cast<size_t>(last[c])].ev = p.events++;

  // copy-outs in job order: small ones on the stream that computed them, the
  // rest on the D2H FIFO after that stream's kernels (piecewise ones after
  // the graph when there is one)
  int waited = -1;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const PlanJob& j = jobs[i];
    const int ks = p.stream_of[i];
    const int job = static_cast<int>(i);
    if (!j.copy_out) {
      if (!graph) op(kOpDone, ks, kend[ks], job);
      continue;
    }
    if (j.local) {
      op(kOpCopyOut, ks, -1, job);
      if (!graph) op(kOpDone, ks, -1, job);
      continue;
    }
    if (graph && j.out_pieces) continue;
    if (waited != ks) {
      op(kOpWait, kPlanD2H, kend[ks]);
      waited = ks;
    }
    op(kOpCopyOut, kPlanD2H, -1, job);
    if (!graph) op(kOpDone, kPlanD2H, -1, job);
  }
  if (!graph) return p;

  // join: every forked stream ends in C0 after its last operation
  for (int s : {kPlanC1, kPlanH2D, kPlanD2H}) op(kOpWait, kPlanC0, record(s));

  // eager, after the launch on C0: the piecewise copy-outs, and the
  // completion of every job
  list = &p.post;
  const int after = record(kPlanC0);
  bool d2h_waits = false;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const PlanJob& j = jobs[i];
    const int job = static_cast<int>(i);
    if (j.copy_out && !j.local && j.out_pieces) {
      if (!d2h_waits) {
        op(kOpWait, kPlanD2H, after);
        d2h_waits = true;
      }
      op(kOpCopyOut, kPlanD2H, -1, job);
      op(kOpDone, kPlanD2H, -1, job);
    } else {
      op(kOpDone, kPlanC0, after, job);
    }
  }
  return p;
}

}  // namespace gvm
