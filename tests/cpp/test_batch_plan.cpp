// CPU check of the grouped batch plan against the rules of streams, events
// and stream capture, restated here independently of the planner:
//  * a stream runs its operations in order; an operation depends on the
//    previous one of its stream and on every event the stream waited for;
//  * an event stands for what its stream had enqueued when it was recorded;
//  * in a capture, only the origin stream (C0) captures at first; another
//    stream joins by waiting for an event recorded on a capturing stream, and
//    every operation must be enqueued on a capturing stream (otherwise it
//    would run once, eagerly, and never be part of the graph);
//  * before the capture ends, every stream that joined must be joined back:
//    C0 waits for an event recorded on it after its last operation.
// Data dependencies checked per job: copy-in -> its launch -> copy-out ->
// completion (eager); a piecewise input (queued on the H2D FIFO before the
// batch) -> its launch.  Exit status 0 when every scenario behaves as stated.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "batch_plan.hpp"
#include "gvm.h"

using namespace gvm;

namespace {

struct Sim {
  struct Node {
    std::set<int> deps;
  };
  std::vector<Node> nodes;
  std::set<int> frontier[kPlanStreams];
  bool capturing[kPlanStreams] = {false, false, false, false};
  int position[kPlanStreams] = {0, 0, 0, 0};  // operations enqueued per stream
  struct Ev {
    std::set<int> nodes;
    int stream = -1, position = -1;
    bool captured = false;
    bool recorded = false;
  };
  std::vector<Ev> ev;
  std::vector<int> joined_at;  // per stream: position of the last event C0 waited for
  std::string error;

  int add_node(int s) {
    nodes.push_back(Node{frontier[s]});
    const int id = static_cast<int>(nodes.size() - 1);
    frontier[s] = {id};
    return id;
  }
  bool ancestor(int a, int d) const {  // a is d or an ancestor of d
    std::vector<int> stack{d};
    std::set<int> seen;
    while (!stack.empty()) {
      const int x = stack.back();
      stack.pop_back();
      if (x == a) return true;
      if (!seen.insert(x).second) continue;
      for (int y : nodes[static_cast<size_t>(x)].deps) stack.push_back(y);
    }
    return false;
  }
  bool covered(int a, const std::set<int>& set) const {
    for (int d : set)
      if (ancestor(a, d)) return true;
    return false;
  }
};

// Replays one operation list.  `capture`: the list is being captured.
struct Replay {
  const BatchPlan& p;
  const std::vector<PlanJob>& jobs;
  Sim sim;
  int pieces_node = -1;
  std::vector<int> in_node, out_node, launch_node, launched, done;
  std::string* why;

  Replay(const BatchPlan& plan, const std::vector<PlanJob>& js, std::string* w)
      : p(plan), jobs(js), in_node(js.size(), -1), out_node(js.size(), -1), launch_node(js.size(), -1),
        launched(js.size(), 0), done(js.size(), 0), why(w) {
    sim.ev.resize(static_cast<size_t>(p.events));
    sim.joined_at.assign(kPlanStreams, -1);
  }

  const char* run(const std::vector<PlanOp>& ops, bool capture) {
    for (const PlanOp& o : ops) {
      if (o.stream < 0 || o.stream >= kPlanStreams) return "bad stream";
      const bool joins = o.kind == kOpWait && o.ev >= 0 && o.ev < p.events && sim.ev[static_cast<size_t>(o.ev)].captured;
      if (capture && !sim.capturing[o.stream] && !joins) {
        *why = "operation kind " + std::to_string(o.kind) + " on stream " + std::to_string(o.stream);
        return "operation on a stream outside the capture";
      }
      sim.position[o.stream]++;
      switch (o.kind) {
        case kOpRecord: {
          if (o.ev < 0 || o.ev >= p.events || sim.ev[static_cast<size_t>(o.ev)].recorded) return "event recorded twice or out of range";
          sim.ev[static_cast<size_t>(o.ev)] = Sim::Ev{sim.frontier[o.stream], o.stream, sim.position[o.stream], sim.capturing[o.stream], true};
          break;
        }
        case kOpWait: {
          if (o.ev < 0 || o.ev >= p.events || !sim.ev[static_cast<size_t>(o.ev)].recorded) return "wait for an event not yet recorded";
          const Sim::Ev& e = sim.ev[static_cast<size_t>(o.ev)];
          if (capture && !sim.capturing[o.stream]) {
            // joining a capture: what the stream ran eagerly before is no
            // dependency of its captured work
            sim.frontier[o.stream] = e.nodes;
            sim.capturing[o.stream] = true;
          } else {
            if (capture != e.captured) return "a wait across the boundary of the capture";
            sim.frontier[o.stream].insert(e.nodes.begin(), e.nodes.end());
          }
          if (o.stream == kPlanC0) sim.joined_at[static_cast<size_t>(e.stream)] = e.position;
          break;
        }
        case kOpCopyIn: {
          const size_t j = static_cast<size_t>(o.job);
          if (o.job < 0 || j >= jobs.size() || !jobs[j].copy_in || jobs[j].pieces || in_node[j] >= 0) return "bad copy-in";
          in_node[j] = sim.add_node(o.stream);
          break;
        }
        case kOpLaunch: {
          if (o.group < 0 || static_cast<size_t>(o.group) >= p.groups.size()) return "bad group";
          const int id = sim.add_node(o.stream);
          for (int j : p.groups[static_cast<size_t>(o.group)].jobs) {
            const size_t u = static_cast<size_t>(j);
            launch_node[u] = id;
            launched[u]++;
            const PlanJob& pj = jobs[u];
            if (pj.copy_in && !pj.pieces && (in_node[u] < 0 || !sim.ancestor(in_node[u], id))) {
              *why = "job " + std::to_string(j);
              return "a launch does not wait for its copy-in";
            }
            if (pj.copy_in && pj.pieces && !sim.ancestor(pieces_node, id)) {
              *why = "job " + std::to_string(j);
              return "a launch does not wait for its piecewise input";
            }
          }
          if (o.ev >= 0) {
            if (o.ev >= p.events || sim.ev[static_cast<size_t>(o.ev)].recorded) return "launch marker recorded twice";
            sim.ev[static_cast<size_t>(o.ev)] = Sim::Ev{sim.frontier[o.stream], o.stream, sim.position[o.stream],
                                                       sim.capturing[o.stream], true};
          }
          break;
        }
        case kOpCopyOut: {
          const size_t j = static_cast<size_t>(o.job);
          if (o.job < 0 || j >= jobs.size() || !jobs[j].copy_out || out_node[j] >= 0) return "bad copy-out";
          out_node[j] = sim.add_node(o.stream);
          if (launch_node[j] < 0 || !sim.ancestor(launch_node[j], out_node[j])) {
            *why = "job " + std::to_string(j);
            return "a copy-out does not wait for its launch";
          }
          break;
        }
        case kOpDone: {
          const size_t j = static_cast<size_t>(o.job);
          if (capture) return "a per-job completion inside a capture";
          if (o.job < 0 || j >= jobs.size()) return "bad completion";
          done[j]++;
          std::set<int> at;
          if (o.ev >= 0) {
            if (o.ev >= p.events || !sim.ev[static_cast<size_t>(o.ev)].recorded) return "completion on an unrecorded event";
            at = sim.ev[static_cast<size_t>(o.ev)].nodes;
          } else {
            at = sim.frontier[o.stream];
          }
          const int last = jobs[j].copy_out ? out_node[j] : launch_node[j];
          if (last < 0 || !sim.covered(last, at)) {
            *why = "job " + std::to_string(j);
            return "a completion does not follow the job's last operation";
          }
          break;
        }
        default:
          return "unknown operation";
      }
    }
    return nullptr;
  }
};

const char* check(const BatchPlan& p, const std::vector<PlanJob>& jobs, bool graph, std::string* why) {
  Replay R(p, jobs, why);
  Sim& sim = R.sim;
  for (size_t g = 0; g < p.groups.size(); ++g) {
    const PlanGroup& G = p.groups[g];
    if (G.jobs.empty() || G.jobs.size() > static_cast<size_t>(kPlanMaxGroup)) return "group size out of range";
    for (size_t i = 0; i < G.jobs.size(); ++i) {
      const PlanJob& j = jobs[static_cast<size_t>(G.jobs[i])];
      if (j.kernel_id != G.kernel_id) return "a group mixes kernels";
      if (G.kernel_id == GVM_K_SGEMM && i > 0 && jobs[static_cast<size_t>(G.jobs[i - 1])].n < j.n)
        return "SGEMM group not largest first";
    }
  }
  bool any_pieces = false;
  for (const PlanJob& j : jobs) any_pieces |= j.pieces && j.copy_in;
  if (any_pieces) R.pieces_node = sim.add_node(kPlanH2D);  // queued before the batch
  const char* err = nullptr;
  if (!graph) {
    if (!p.pre.empty() || !p.post.empty()) return "an eager batch with pre or post operations";
    err = R.run(p.ops, false);
  } else {
    err = R.run(p.pre, false);
    if (err) return err;
    // the capture: C0 starts it; captured work is on no stream afterwards
    std::set<int> saved[kPlanStreams];
    for (int s = 0; s < kPlanStreams; ++s) saved[s] = sim.frontier[s];
    const size_t first = sim.nodes.size();
    const int pos0[kPlanStreams] = {sim.position[0], sim.position[1], sim.position[2], sim.position[3]};
    sim.capturing[kPlanC0] = true;
    err = R.run(p.ops, true);
    if (err) return err;
    for (int s = 1; s < kPlanStreams; ++s) {
      if (!sim.capturing[s] || sim.position[s] == pos0[s]) continue;
      if (sim.joined_at[static_cast<size_t>(s)] != sim.position[s]) {
        *why = "stream " + std::to_string(s) + " has " + std::to_string(sim.position[s] - pos0[s]) +
               " captured operations, joined after " + std::to_string(sim.joined_at[static_cast<size_t>(s)] - pos0[s]);
        return "a stream forked into the capture is not joined after its last operation";
      }
    }
    for (int s = 0; s < kPlanStreams; ++s) {
      sim.capturing[s] = false;
      sim.frontier[s] = saved[s];
    }
    // the graph launch on C0: after C0's eager work, and containing every captured node
    std::set<int> deps = saved[kPlanC0];
    for (size_t x = first; x < sim.nodes.size(); ++x) deps.insert(static_cast<int>(x));
    sim.nodes.push_back(Sim::Node{deps});
    sim.frontier[kPlanC0] = {static_cast<int>(sim.nodes.size() - 1)};
    err = R.run(p.post, false);
  }
  if (err) return err;
  for (size_t j = 0; j < jobs.size(); ++j) {
    if (R.launched[j] != 1) return "a job is not launched exactly once";
    if (jobs[j].copy_out && R.out_node[j] < 0) return "a copy-out is missing";
    if (jobs[j].copy_in && !jobs[j].pieces && R.in_node[j] < 0) return "a copy-in is missing";
    if (R.done[j] != 1) return "a job has no single completion";
  }
  return nullptr;
}

PlanJob job(int k, uint64_t n, bool in, bool out, bool pieces = false) {
  uint64_t in_b = 0, out_b = 0;
  switch (k) {
    case GVM_K_VECADD: case GVM_K_VECMUL: in_b = 8 * n; out_b = 4 * n; break;
    case GVM_K_BLACKSCHOLES: in_b = 12 * n; out_b = 8 * n; break;
    case GVM_K_SGEMM: in_b = 8 * n * n; out_b = 4 * n * n; break;
    default: in_b = 16; out_b = 96; break;
  }
  const bool local = (in ? in_b : 0) + (out ? out_b : 0) <= (1u << 20);
  return PlanJob{k, n, in, out, local, pieces && in && !local, pieces && out && !local};
}

int failures = 0;

// Every launch order: both compute streams longest first, one stream longest
// first, one stream shortest first.
void expect_ok(const char* name, const std::vector<PlanJob>& jobs, bool graph) {
  const int streams[3] = {2, 1, 1};
  const bool longest[3] = {true, true, false};
  for (int v = 0; v < 3; ++v) {
    std::string why;
    const BatchPlan p = plan_grouped(jobs, graph, streams[v], longest[v]);
    const char* err = check(p, jobs, graph, &why);
    if (err) {
      if (++failures > 20) return;
      printf("FAIL %s (%s, order %d): %s %s\n", name, graph ? "graph" : "eager", v, err, why.c_str());
    }
  }
}

}  // namespace

int main() {
  // the mix of the graph replay test: vector add 300001 (copies on the
  // FIFOs), Black-Scholes 50001 and SGEMM 192 (local copies); Black-Scholes
  // is dealt to compute stream 1
  std::vector<PlanJob> mix;
  for (int r = 0; r < 6; ++r) {
    const int k = r % 3 + 1;
    mix.push_back(job(k, k == 1 ? 300001 : k == 2 ? 50001 : 192, true, true));
  }
  expect_ok("graph test mix", mix, true);
  expect_ok("graph test mix", mix, false);

  // the earlier capture schedule, restated: compute stream 1 was joined
  // right after its kernels, before the local copy-outs queued behind them
  {
    const BatchPlan good = plan_grouped(mix, true);
    BatchPlan old = good;
    old.ops.clear();
    // drop the final join of C1 (record on C1, C0 waits) ...
    int join_ev = -1;
    for (size_t i = 0; i + 1 < good.ops.size(); ++i)
      if (good.ops[i].kind == kOpRecord && good.ops[i].stream == kPlanC1 && good.ops[i + 1].kind == kOpWait &&
          good.ops[i + 1].stream == kPlanC0 && i + 6 >= good.ops.size())
        join_ev = good.ops[i].ev;
    if (join_ev < 0) {
      ++failures;
      printf("FAIL: no final join of compute stream 1 in the capture plan\n");
    }
    for (const PlanOp& o : good.ops) {
      if (o.ev == join_ev && (o.kind == kOpRecord || o.kind == kOpWait)) continue;
      old.ops.push_back(o);
      // ... and join C1 at its kernel-end marker instead, as before
      if (o.kind == kOpLaunch && o.ev >= 0 && o.stream == kPlanC1) {
        old.ops.push_back(PlanOp{kOpRecord, kPlanC1, join_ev, -1, -1});
        old.ops.push_back(PlanOp{kOpWait, kPlanC0, join_ev, -1, -1});
      }
    }
    std::string why;
    const char* err = check(old, mix, true, &why);
    if (!err || std::string(err).find("not joined") == std::string::npos) {
      ++failures;
      printf("FAIL: the early join of compute stream 1 was not detected (%s)\n", err ? err : "accepted");
    } else {
      printf("early join detected: %s (%s)\n", err, why.c_str());
    }
  }

  // a compute stream that does not wait for the H2D FIFO reads its inputs too early
  {
    std::vector<PlanJob> two{job(GVM_K_VECADD, 300001, true, true), job(GVM_K_BLACKSCHOLES, 100001, true, true)};
    const BatchPlan good = plan_grouped(two, false);
    BatchPlan bad = good;
    bad.ops.clear();
    bool dropped = false;
    for (size_t i = 0; i < good.ops.size(); ++i) {
      const PlanOp& o = good.ops[i];
      if (!dropped && o.kind == kOpWait && o.stream == kPlanC1 && i > 0 && good.ops[i - 1].kind == kOpWait &&
          good.ops[i - 1].stream == kPlanC0) {
        dropped = true;
        continue;
      }
      bad.ops.push_back(o);
    }
    std::string why;
    const char* err = check(bad, two, false, &why);
    expect_ok("vecadd + Black-Scholes over the FIFOs", two, false);
    if (!dropped || !err || std::string(err).find("copy-in") == std::string::npos) {
      ++failures;
      printf("FAIL: a missing wait for the H2D FIFO was not detected (%s)\n", err ? err : "accepted");
    } else {
      printf("missing input wait detected: %s (%s)\n", err, why.c_str());
    }
  }

  // every shape of batch: random mixes of kernels, sizes and copy flags
  std::mt19937_64 rng(1511);
  const int kernels[] = {GVM_K_VECADD, GVM_K_BLACKSCHOLES, GVM_K_SGEMM, GVM_K_VECMUL, GVM_K_EP};
  for (int t = 0; t < 4000; ++t) {
    const int nj = 1 + static_cast<int>(rng() % 70);
    std::vector<PlanJob> jobs;
    for (int i = 0; i < nj; ++i) {
      const int k = kernels[rng() % 5];
      uint64_t n = 1 + rng() % (k == GVM_K_SGEMM ? 2048 : (1u << 22));
      if (k == GVM_K_SGEMM && rng() % 2) n = 64 * (4 + rng() % 29);
      const bool in = rng() % 4 != 0, out = rng() % 4 != 0;
      jobs.push_back(job(k, n, in, out, rng() % 2 == 0));
    }
    std::vector<PlanJob> whole = jobs;
    for (auto& j : whole) j.pieces = j.out_pieces = false;
    expect_ok("random whole copies", whole, true);
    expect_ok("random whole copies", whole, false);
    expect_ok("random pieces", jobs, true);
    expect_ok("random pieces", jobs, false);
  }
  // the 32-rank uneven batch: 16 vector adds and 16 SGEMMs, copies in pieces
  {
    const uint64_t vec[] = {13474670, 2746283, 151966, 260220, 877892, 302835, 14520833, 11550894,
                            76752, 324147, 9554722, 72333, 11775798, 1539844, 174914, 491127};
    const uint64_t gemm[] = {704, 1280, 960, 384, 1728, 1216, 1216, 1920, 704, 448, 832, 1408, 704, 1664, 832, 1280};
    std::vector<PlanJob> c4;
    for (uint64_t n : vec) c4.push_back(job(GVM_K_VECADD, n, true, true, true));
    for (uint64_t n : gemm) c4.push_back(job(GVM_K_SGEMM, n, true, true, true));
    expect_ok("uneven 32-rank batch", c4, true);
    expect_ok("uneven 32-rank batch", c4, false);
    // a graph launched without first waiting for the input pieces
    BatchPlan bad = plan_grouped(c4, true);
    const size_t had = bad.pre.size();
    bad.pre.clear();
    std::string why;
    const char* err = check(bad, c4, true, &why);
    if (had == 0 || !err || std::string(err).find("piecewise input") == std::string::npos) {
      ++failures;
      printf("FAIL: a graph that does not wait for the input pieces was not detected (%s)\n", err ? err : "accepted");
    } else {
      printf("graph without the input wait detected: %s (%s)\n", err, why.c_str());
    }
  }
  // one kernel kind only (one group, compute stream 1 idle), and 33 requests of one kernel (two groups)
  expect_ok("single", {job(GVM_K_SGEMM, 1024, true, true)}, true);
  expect_ok("single", {job(GVM_K_SGEMM, 1024, true, true)}, false);
  std::vector<PlanJob> many(33, job(GVM_K_VECADD, 1 << 20, true, true));
  expect_ok("33 of one kernel", many, true);
  expect_ok("33 of one kernel", many, false);
  std::vector<PlanJob> resident(8, job(GVM_K_SGEMM, 1024, false, false));
  expect_ok("resident", resident, true);
  expect_ok("resident", resident, false);

  printf("%s: %d failures\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
